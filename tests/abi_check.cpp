// abi_check.cpp -- drives every entry point of the C ABI (include/sdq.h)
// from C++, for a build of the host runtime with AddressSanitizer and
// UndefinedBehaviorSanitizer: any out-of-bounds access, use after free,
// leak or undefined behaviour in the runtime's argument checks, planning,
// checkpoint handles, graph cache, profiling tables or autotune cache aborts
// the run.  Numerical parity is the business of the Python tests; here each
// call must succeed (or fail with the documented status), leave finite
// outputs, and agree with the other calls that compute the same quantity.
//
// Without a usable device (no GPU) only the paths that need none run: a
// failing sdq_create, NULL contexts, version and error strings.
// Exit status 0 = every check passed; the last line printed says how many.
#include <hip/hip_runtime.h>

#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include <unistd.h>

#include "sdq.h"

namespace {

int g_checks = 0;

void check(bool ok, const char* what, const char* file, int line) {
  ++g_checks;
  if (!ok) {
    fprintf(stderr, "abi_check: FAILED %s (%s:%d)\n", what, file, line);
    fflush(stderr);
    exit(1);
  }
}
#define CHECK(c) check((c), #c, __FILE__, __LINE__)
#define HIPCHECK(c) check((c) == hipSuccess, #c, __FILE__, __LINE__)

// splitmix64: a small counter-free stream of seeded numbers for the inputs
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  double unif() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
  double normal() {  // Box-Muller
    double u1 = unif(), u2 = unif();
    if (u1 < 1e-300) u1 = 1e-300;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
  }
};

// hopping matrix of an L x L periodic square lattice (t = 1)
std::vector<double> hopping(int L) {
  const int n = L * L;
  std::vector<double> K((size_t)n * n, 0.0);
  for (int x = 0; x < L; ++x)
    for (int y = 0; y < L; ++y) {
      const int i = x * L + y;
      const int nb[2] = {((x + 1) % L) * L + y, x * L + (y + 1) % L};
      for (int j : nb) {
        K[(size_t)i * n + j] -= 1.0;
        K[(size_t)j * n + i] -= 1.0;
      }
    }
  return K;
}

// exp(s K) by its Taylor series (|s| ||K|| <= 0.4 here, 30 terms)
std::vector<double> expm(const std::vector<double>& K, int n, double s) {
  std::vector<double> E((size_t)n * n, 0.0), T((size_t)n * n, 0.0), U((size_t)n * n);
  for (int i = 0; i < n; ++i) E[(size_t)i * n + i] = T[(size_t)i * n + i] = 1.0;
  for (int j = 1; j <= 30; ++j) {
    for (int r = 0; r < n; ++r)
      for (int c = 0; c < n; ++c) {
        double acc = 0.0;
        for (int q = 0; q < n; ++q) acc += T[(size_t)r * n + q] * K[(size_t)q * n + c];
        U[(size_t)r * n + c] = acc * s / j;
      }
    T.swap(U);
    for (size_t e = 0; e < E.size(); ++e) E[e] += T[e];
  }
  return E;
}

// device buffers freed at exit of the scope
struct Dev {
  std::vector<void*> ptrs;
  template <class T>
  T* alloc(size_t count) {
    void* p = nullptr;
    HIPCHECK(hipMalloc(&p, (count ? count : 1) * sizeof(T)));
    HIPCHECK(hipMemset(p, 0, (count ? count : 1) * sizeof(T)));
    ptrs.push_back(p);
    return static_cast<T*>(p);
  }
  template <class T>
  T* upload(const std::vector<T>& h) {
    T* p = alloc<T>(h.size());
    HIPCHECK(hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
  }
  ~Dev() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

template <class T>
std::vector<T> down(const T* d, size_t count) {
  std::vector<T> h(count);
  HIPCHECK(hipMemcpy(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost));
  return h;
}

bool all_finite(const std::vector<double>& v) {
  for (double x : v)
    if (!std::isfinite(x)) return false;
  return true;
}

double rel_diff(const std::vector<double>& a, const std::vector<double>& b) {
  double num = 0.0, den = 0.0;
  for (size_t i = 0; i < a.size(); ++i) {
    num += (a[i] - b[i]) * (a[i] - b[i]);
    den += b[i] * b[i];
  }
  return std::sqrt(num / (den > 0 ? den : 1.0));
}

// one lattice: the slice exponentials on the device
struct Lattice {
  int L, n;
  double* expk;
  double* expk_inv;
  std::vector<double> h_expk;
};

Lattice lattice(Dev& dev, int L, double dtau) {
  Lattice lat;
  lat.L = L;
  lat.n = L * L;
  const std::vector<double> K = hopping(L);
  lat.h_expk = expm(K, lat.n, -dtau);
  lat.expk = dev.upload(lat.h_expk);
  lat.expk_inv = dev.upload(expm(K, lat.n, dtau));
  return lat;
}

std::vector<double> ising_field(Rng& r, int m, int n) {
  std::vector<double> f((size_t)m * n);
  for (double& x : f) x = r.unif() < 0.5 ? -1.0 : 1.0;
  return f;
}

std::vector<double> gauss_field(Rng& r, int m, int n, double sd) {
  std::vector<double> f((size_t)m * n);
  for (double& x : f) x = sd * r.normal();
  return f;
}

void no_device_paths() {
  // every compute entry point on a NULL context is an argument error
  sdq_instance inst{};
  double* p = nullptr;
  CHECK(sdq_greens(nullptr, &inst, 1, SDQ_INV_LOH, &p, nullptr, nullptr, nullptr) == SDQ_EINVAL);
  CHECK(sdq_greens_noalloc(nullptr, &inst, 1, SDQ_INV_LOH, &p, nullptr, nullptr, nullptr) == SDQ_EINVAL);
  CHECK(sdq_greens_tdisp(nullptr, &inst, 1, SDQ_INV_LOH, nullptr, 0, &p, &p, nullptr, nullptr, nullptr) ==
        SDQ_EINVAL);
  CHECK(sdq_logdet(nullptr, &inst, 1, nullptr, nullptr, nullptr, nullptr) == SDQ_EINVAL);
  CHECK(sdq_logdet_grad(nullptr, 0, &inst, 1, &p, nullptr, nullptr, nullptr) == SDQ_EINVAL);
  CHECK(sdq_release(nullptr, 1) == SDQ_EINVAL);
  CHECK(sdq_udt(nullptr, 4, 1, nullptr, nullptr, nullptr, nullptr) == SDQ_EINVAL);
  CHECK(sdq_udt_complex(nullptr, 4, 1, nullptr, nullptr, nullptr, nullptr) == SDQ_EINVAL);
  CHECK(sdq_set_stabilizer(nullptr, SDQ_STAB_QR) == SDQ_EINVAL);
  CHECK(sdq_set_graphs(nullptr, 1) == SDQ_EINVAL);
  CHECK(sdq_set_profiling(nullptr, 1) == SDQ_EINVAL);
  CHECK(sdq_sync(nullptr) == SDQ_EINVAL);
  CHECK(sdq_tune(nullptr, nullptr, 0, nullptr) == SDQ_EINVAL);
  int64_t launches = 0;
  double ms = 0.0;
  CHECK(sdq_kernel_stats(nullptr, "sweep", &launches, &ms) == SDQ_EINVAL);
  char buf[8];
  CHECK(sdq_kernel_names(nullptr, buf, sizeof buf) == SDQ_EINVAL);
  const char* e = sdq_last_error(nullptr);
  CHECK(e != nullptr);
  sdq_destroy(nullptr);
  CHECK(sdq_version() != nullptr && strlen(sdq_version()) > 0);
}

void with_device(sdq_ctx* ctx) {
  Dev dev;
  Rng rng{20031105};
  const double dtau = 0.1, U = 4.0;
  const double lambda = std::acosh(std::exp(0.5 * dtau * U));
  const int m = 40, k = 10;

  // equal-time G of a mixed batch: both kernel families (n <= 128 one
  // workgroup, n = 144 one workgroup with device-memory factors, n = 169 gang)
  const int Ls[] = {4, 6, 10, 12, 13, 4};
  const int nc = 6;
  std::vector<Lattice> lats;
  std::vector<sdq_instance> inst(nc);
  std::vector<double*> g(nc), gt(nc), g2(nc);
  const int l_list[] = {0, 5, 10, 40};
  const int n_l = 4;
  for (int c = 0; c < nc; ++c) {
    lats.push_back(lattice(dev, Ls[c], dtau));
    const int n = lats[c].n;
    inst[c] = sdq_instance{};
    inst[c].n = n;
    inst[c].m = m;
    inst[c].k = (c == 5) ? 7 : k;  // a ragged last block
    inst[c].expk = lats[c].expk;
    inst[c].expk_inv = lats[c].expk_inv;
    inst[c].field = dev.upload(ising_field(rng, m, n));
    inst[c].alpha = (c % 2) ? -lambda : lambda;
    g[c] = dev.alloc<double>((size_t)n * n);
    g2[c] = dev.alloc<double>((size_t)n * n);
    gt[c] = dev.alloc<double>((size_t)n_l * n * n);
  }
  double* ld = dev.alloc<double>(nc);
  double* sg = dev.alloc<double>(nc);
  int32_t* st = dev.alloc<int32_t>(nc);
  double* ld2 = dev.alloc<double>(nc);
  double* sg2 = dev.alloc<double>(nc);
  int32_t* st2 = dev.alloc<int32_t>(nc);

  CHECK(sdq_set_profiling(ctx, 1) == SDQ_OK);
  CHECK(sdq_greens(ctx, inst.data(), nc, SDQ_INV_LOH, g.data(), ld, sg, st) == SDQ_OK);
  CHECK(sdq_sync(ctx) == SDQ_OK);
  const std::vector<double> h_ld = down(ld, nc);
  for (int s : down(st, nc)) CHECK(s == SDQ_OK);
  CHECK(all_finite(h_ld));
  std::vector<std::vector<double>> h_g(nc);
  for (int c = 0; c < nc; ++c) {
    h_g[c] = down(g[c], (size_t)inst[c].n * inst[c].n);
    CHECK(all_finite(h_g[c]));
  }

  // the same batch again with graphs: capture, then replay, equal results
  CHECK(sdq_set_graphs(ctx, 1) == SDQ_OK);
  for (int rep = 0; rep < 2; ++rep) {
    CHECK(sdq_greens(ctx, inst.data(), nc, SDQ_INV_LOH, g2.data(), ld2, sg2, st2) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    for (int c = 0; c < nc; ++c)
      CHECK(rel_diff(down(g2[c], (size_t)inst[c].n * inst[c].n), h_g[c]) == 0.0);
  }
  CHECK(sdq_set_graphs(ctx, 0) == SDQ_OK);

  // time-displaced: its equal-time G and log det agree with sdq_greens
  CHECK(sdq_greens_tdisp(ctx, inst.data(), nc, SDQ_INV_LOH, l_list, n_l, gt.data(), g2.data(), ld2, sg2, st2) ==
        SDQ_OK);
  CHECK(sdq_sync(ctx) == SDQ_OK);
  for (int s : down(st2, nc)) CHECK(s == SDQ_OK);
  const std::vector<double> h_ld2 = down(ld2, nc);
  for (int c = 0; c < nc; ++c) {
    const size_t nn = (size_t)inst[c].n * inst[c].n;
    CHECK(rel_diff(down(g2[c], nn), h_g[c]) < 1e-10);
    CHECK(std::fabs(h_ld2[c] - h_ld[c]) <= 1e-10 * std::fabs(h_ld[c]) + 1e-12);
    const std::vector<double> h_gt = down(gt[c], n_l * nn);
    CHECK(all_finite(h_gt));
    // G(0, 0) = G
    CHECK(rel_diff(std::vector<double>(h_gt.begin(), h_gt.begin() + nn), h_g[c]) < 1e-10);
  }

  // the plain scheme on the one-workgroup sizes
  {
    std::vector<sdq_instance> small(inst.begin(), inst.begin() + 3);
    CHECK(sdq_greens_tdisp(ctx, small.data(), 3, SDQ_INV_PLAIN, l_list, n_l, gt.data(), g2.data(), nullptr,
                           nullptr, st2) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    for (int s : down(st2, 3)) CHECK(s == SDQ_OK);
  }

  // log det with a checkpoint, the gradient from it, and without one
  std::vector<double*> grad(nc), grad2(nc);
  for (int c = 0; c < nc; ++c) {
    grad[c] = dev.alloc<double>((size_t)m * inst[c].n);
    grad2[c] = dev.alloc<double>((size_t)m * inst[c].n);
  }
  uint64_t handle = 0;
  CHECK(sdq_logdet(ctx, inst.data(), nc, ld2, sg2, st2, &handle) == SDQ_OK);
  CHECK(handle != 0);
  CHECK(sdq_logdet_grad(ctx, handle, inst.data(), nc, grad.data(), nullptr, nullptr, st2) == SDQ_OK);
  CHECK(sdq_release(ctx, handle) == SDQ_OK);
  CHECK(sdq_release(ctx, handle) == SDQ_EINVAL);  // released once only
  CHECK(sdq_logdet_grad(ctx, 0, inst.data(), nc, grad2.data(), ld2, sg2, st2) == SDQ_OK);
  CHECK(sdq_sync(ctx) == SDQ_OK);
  for (int s : down(st2, nc)) CHECK(s == SDQ_OK);
  for (int c = 0; c < nc; ++c) {
    const std::vector<double> a = down(grad[c], (size_t)m * inst[c].n);
    CHECK(all_finite(a));
    CHECK(rel_diff(down(grad2[c], (size_t)m * inst[c].n), a) < 1e-10);
  }
  // a handle left for sdq_destroy to release
  uint64_t kept = 0;
  CHECK(sdq_logdet(ctx, inst.data(), 2, ld2, sg2, st2, &kept) == SDQ_OK);

  // the allocation-free entry point on the n <= 128 chains
  {
    std::vector<sdq_instance> small(inst.begin(), inst.begin() + 3);
    CHECK(sdq_greens_noalloc(ctx, small.data(), 3, SDQ_INV_LOH, g2.data(), ld2, sg2, st2) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    for (int c = 0; c < 3; ++c)
      CHECK(rel_diff(down(g2[c], (size_t)inst[c].n * inst[c].n), h_g[c]) < 1e-12);
    CHECK(sdq_greens_noalloc(ctx, inst.data(), nc, SDQ_INV_LOH, g2.data(), ld2, sg2, st2) ==
          SDQ_EUNSUPPORTED);  // n > 128 in the batch
  }

  // the Jacobi SVD stabilizer on n <= 80, then back to the QR
  {
    CHECK(sdq_set_stabilizer(ctx, SDQ_STAB_SVD) == SDQ_OK);
    CHECK(sdq_greens(ctx, inst.data(), 2, SDQ_INV_LOH, g2.data(), ld2, sg2, st2) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    for (int c = 0; c < 2; ++c)
      CHECK(rel_diff(down(g2[c], (size_t)inst[c].n * inst[c].n), h_g[c]) < 1e-10);
    CHECK(sdq_greens(ctx, inst.data(), nc, SDQ_INV_LOH, g2.data(), ld2, sg2, st2) == SDQ_EUNSUPPORTED);
    CHECK(sdq_set_stabilizer(ctx, SDQ_STAB_QR) == SDQ_OK);
    CHECK(sdq_set_stabilizer(ctx, 7) == SDQ_EINVAL);
  }

  // dense slices B_l = expk diag(exp(alpha f_l)) equal the structured chain
  {
    const int c = 1, n = inst[c].n;
    const std::vector<double> f = down(inst[c].field, (size_t)m * n);
    std::vector<double> sl((size_t)m * n * n);
    for (int l = 0; l < m; ++l)
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          sl[((size_t)l * n + i) * n + j] = lats[c].h_expk[(size_t)i * n + j] * std::exp(inst[c].alpha * f[(size_t)l * n + j]);
    sdq_dense_instance di{};
    di.n = n;
    di.m = m;
    di.k = k;
    di.slices = dev.upload(sl);
    double* gd = dev.alloc<double>((size_t)n * n);
    double* gtd = dev.alloc<double>((size_t)n_l * n * n);
    CHECK(sdq_greens_dense(ctx, &di, 1, &gd, ld2, sg2, st2) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    CHECK(rel_diff(down(gd, (size_t)n * n), h_g[c]) < 1e-10);
    CHECK(sdq_greens_tdisp_dense(ctx, &di, 1, l_list, n_l, &gtd, &gd, ld2, sg2, st2) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    const std::vector<double> a = down(gtd, (size_t)n_l * n * n);
    const std::vector<double> b = down(gt[c], (size_t)n_l * n * n);
    CHECK(rel_diff(a, b) < 1e-10);
    const int bad_list[] = {5, 0};
    CHECK(sdq_greens_tdisp_dense(ctx, &di, 1, bad_list, 2, &gtd, &gd, ld2, sg2, st2) == SDQ_EINVAL);
  }

  // complex slices: real slices in complex form agree with the real chain
  {
    const int c = 0, n = inst[c].n;
    const std::vector<double> f = down(inst[c].field, (size_t)m * n);
    std::vector<double> sl((size_t)2 * m * n * n, 0.0);
    for (int l = 0; l < m; ++l)
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
          sl[2 * (((size_t)l * n + i) * n + j)] =
              lats[c].h_expk[(size_t)i * n + j] * std::exp(inst[c].alpha * f[(size_t)l * n + j]);
    sdq_complex_instance ci{};
    ci.n = n;
    ci.m = m;
    ci.k = k;
    ci.slices = dev.upload(sl);
    double* gc = dev.alloc<double>((size_t)2 * n * n);
    double* ph = dev.alloc<double>(2);
    CHECK(sdq_greens_complex(ctx, &ci, 1, &gc, ld2, ph, st2) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    const std::vector<double> z = down(gc, (size_t)2 * n * n);
    std::vector<double> re((size_t)n * n);
    for (size_t e = 0; e < re.size(); ++e) re[e] = z[2 * e];
    CHECK(rel_diff(re, h_g[c]) < 1e-10);
    ci.n = 65;
    CHECK(sdq_greens_complex(ctx, &ci, 1, &gc, ld2, ph, st2) == SDQ_EUNSUPPORTED);
  }

  // UDT of plain matrices (one workgroup and gang sizes) and complex ones
  for (int n : {20, 150}) {
    const int cnt = (n > 128) ? 2 : 64;
    std::vector<double> w((size_t)cnt * n * n);
    for (double& x : w) x = rng.normal();
    const double* dw = dev.upload(w);
    double* u = dev.alloc<double>((size_t)cnt * n * n);
    double* d = dev.alloc<double>((size_t)cnt * n);
    double* t = dev.alloc<double>((size_t)cnt * n * n);
    CHECK(sdq_udt(ctx, n, cnt, dw, u, d, t) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    CHECK(all_finite(down(u, (size_t)cnt * n * n)) && all_finite(down(t, (size_t)cnt * n * n)));
  }
  {
    const int n = 20, cnt = 16;
    std::vector<double> w((size_t)2 * cnt * n * n);
    for (double& x : w) x = rng.normal();
    const double* dw = dev.upload(w);
    double* u = dev.alloc<double>((size_t)2 * cnt * n * n);
    double* d = dev.alloc<double>((size_t)cnt * n);
    double* t = dev.alloc<double>((size_t)2 * cnt * n * n);
    CHECK(sdq_udt_complex(ctx, n, cnt, dw, u, d, t) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    CHECK(all_finite(down(d, (size_t)cnt * n)));
    CHECK(sdq_udt_complex(ctx, 65, cnt, dw, u, d, t) == SDQ_EUNSUPPORTED);
    CHECK(sdq_udt_complex(ctx, n, -1, dw, u, d, t) == SDQ_EINVAL);
  }

  // the chain's UDT factors (chains of one n)
  {
    const int n = inst[0].n;
    sdq_instance two[2] = {inst[0], inst[5]};
    double* u = dev.alloc<double>((size_t)2 * n * n);
    double* d = dev.alloc<double>((size_t)2 * n);
    double* t = dev.alloc<double>((size_t)2 * n * n);
    CHECK(sdq_chain_udt(ctx, two, 2, u, d, t) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    CHECK(all_finite(down(d, (size_t)2 * n)));
  }

  // the symmetric slice form's similarity transform
  {
    const int n = inst[0].n;
    double* mats[2] = {g2[0], g2[5]};
    CHECK(sdq_similarity(ctx, n, 2, lats[0].expk_inv, lats[0].expk, mats) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    CHECK(sdq_similarity(ctx, 129, 2, lats[0].expk_inv, lats[0].expk, mats) == SDQ_EUNSUPPORTED);
  }

  // Monte Carlo drivers: two chains of two flavours (alpha = +-lambda)
  const int cnt = 2, nf = 2;
  std::vector<sdq_instance> mc(cnt * nf), prop(cnt * nf);
  for (int c = 0; c < cnt; ++c) {
    const Lattice& lat = lats[c];  // n = 16 and 36
    double* f = dev.upload(ising_field(rng, m, lat.n));
    double* fp = dev.upload(ising_field(rng, m, lat.n));
    for (int fl = 0; fl < nf; ++fl) {
      sdq_instance& I = mc[c * nf + fl];
      I = sdq_instance{};
      I.n = lat.n;
      I.m = m;
      I.k = k;
      I.expk = lat.expk;
      I.expk_inv = lat.expk_inv;
      I.field = f;
      I.alpha = fl ? -lambda : lambda;
      prop[c * nf + fl] = I;
      prop[c * nf + fl].field = fp;
    }
  }
  double* mld = dev.alloc<double>(cnt * nf);
  double* msg = dev.alloc<double>(cnt * nf);
  int32_t* mst = dev.alloc<int32_t>(cnt * nf);
  int32_t* acc = dev.alloc<int32_t>(cnt);
  {
    std::vector<double> un((size_t)cnt * m * 36);
    for (double& x : un) x = rng.unif();
    CHECK(sdq_local_sweep(ctx, mc.data(), cnt, nf, dev.upload(un), acc, mst) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    for (int s : down(mst, cnt * nf)) CHECK(s == SDQ_OK);
    CHECK(sdq_local_sweep(ctx, mc.data(), cnt, 3, dev.upload(un), acc, mst) == SDQ_EINVAL);
  }
  {
    CHECK(sdq_logdet(ctx, mc.data(), cnt * nf, mld, msg, mst, nullptr) == SDQ_OK);
    const double* dS = dev.upload(std::vector<double>(cnt, 0.0));
    const double* u = dev.upload(std::vector<double>{0.3, 0.7});
    CHECK(sdq_metropolis(ctx, mc.data(), prop.data(), cnt, nf, dS, u, mld, msg, acc, mst) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    for (int s : down(mst, cnt * nf)) CHECK(s == SDQ_OK);
    CHECK(all_finite(down(mld, cnt * nf)));
  }
  {
    // continuous field: alpha = dtau g
    std::vector<sdq_instance> cf = mc;
    for (int c = 0; c < cnt; ++c) {
      double* f = dev.upload(gauss_field(rng, m, cf[c * nf].n, 0.5));
      for (int fl = 0; fl < nf; ++fl) {
        cf[c * nf + fl].field = f;
        cf[c * nf + fl].alpha = fl ? -0.1 : 0.1;
      }
    }
    size_t tot = 0;
    for (int c = 0; c < cnt; ++c) tot += (size_t)m * cf[c * nf].n;
    std::vector<double> noise(tot);
    for (double& x : noise) x = rng.normal();
    double* force = dev.alloc<double>(tot);
    CHECK(sdq_langevin(ctx, cf.data(), cnt, nf, 0.01, 1.0, dev.upload(noise), force, mld, msg, mst) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    for (int s : down(mst, cnt * nf)) CHECK(s == SDQ_OK);
    CHECK(all_finite(down(force, tot)));
    for (double& x : noise) x = rng.normal();
    double* dH = dev.alloc<double>(cnt);
    const double* u = dev.upload(std::vector<double>{0.5, 0.5});
    CHECK(sdq_hmc(ctx, cf.data(), cnt, nf, 0.02, 2, 1.0, dev.upload(noise), u, mld, msg, acc, dH, mst) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    for (int s : down(mst, cnt * nf)) CHECK(s == SDQ_OK);
    CHECK(all_finite(down(dH, cnt)));
    CHECK(sdq_hmc(ctx, cf.data(), cnt, nf, 0.02, 0, 1.0, dev.upload(noise), u, mld, msg, acc, dH, mst) ==
          SDQ_EINVAL);
  }

  // the profiling tables
  {
    int64_t launches = 0;
    double ms = 0.0;
    CHECK(sdq_kernel_stats(ctx, "sweep", &launches, &ms) == SDQ_OK);
    CHECK(launches > 0 && ms > 0.0);
    std::vector<char> names(8192);
    CHECK(sdq_kernel_names(ctx, names.data(), (int32_t)names.size()) == SDQ_OK);
    CHECK(strstr(names.data(), "sweep") != nullptr);
    char tiny[2];
    CHECK(sdq_kernel_names(ctx, tiny, sizeof tiny) == SDQ_EINVAL);
    CHECK(sdq_set_profiling(ctx, 0) == SDQ_OK);
  }

  // the autotune table: time n = 16 and 36, write the cache, read it back
  {
    char path[96];
    snprintf(path, sizeof path, "/tmp/sdq_abi_check_tune_%d.jsonl", (int)getpid());
    remove(path);
    const int32_t ns[] = {16, 36, 200};
    CHECK(sdq_tune(ctx, ns, 3, path) == SDQ_OK);
    CHECK(sdq_tune(ctx, ns, 2, path) == SDQ_OK);
    CHECK(sdq_greens(ctx, inst.data(), 2, SDQ_INV_LOH, g2.data(), ld2, sg2, st2) == SDQ_OK);
    CHECK(sdq_sync(ctx) == SDQ_OK);
    for (int c = 0; c < 2; ++c)
      CHECK(rel_diff(down(g2[c], (size_t)inst[c].n * inst[c].n), h_g[c]) < 1e-12);
    remove(path);
  }

  // argument errors: each names itself in sdq_last_error
  {
    sdq_instance bad = inst[0];
    CHECK(sdq_greens(ctx, inst.data(), -1, SDQ_INV_LOH, g.data(), ld, sg, st) == SDQ_EINVAL);
    CHECK(sdq_greens(ctx, nullptr, 1, SDQ_INV_LOH, g.data(), ld, sg, st) == SDQ_EINVAL);
    bad.k = 0;
    CHECK(sdq_greens(ctx, &bad, 1, SDQ_INV_LOH, g.data(), ld, sg, st) == SDQ_EINVAL);
    CHECK(strlen(sdq_last_error(ctx)) > 0);
    bad = inst[0];
    bad.n = 2000;
    CHECK(sdq_greens(ctx, &bad, 1, SDQ_INV_LOH, g.data(), ld, sg, st) == SDQ_EUNSUPPORTED);
    bad = inst[0];
    bad.expk_inv = nullptr;
    CHECK(sdq_logdet_grad(ctx, 0, &bad, 1, grad.data(), ld, sg, st) == SDQ_EINVAL);
    bad = inst[0];
    bad.alpha = NAN;
    CHECK(sdq_greens(ctx, &bad, 1, SDQ_INV_LOH, g.data(), ld, sg, st) == SDQ_EINVAL);
    const int desc[] = {10, 5};
    CHECK(sdq_greens_tdisp(ctx, inst.data(), 1, SDQ_INV_LOH, desc, 2, gt.data(), g.data(), ld, sg, st) ==
          SDQ_EINVAL);
    const int beyond[] = {0, 41};
    CHECK(sdq_greens_tdisp(ctx, inst.data(), 1, SDQ_INV_LOH, beyond, 2, gt.data(), g.data(), ld, sg, st) ==
          SDQ_EINVAL);
    CHECK(sdq_greens(ctx, inst.data(), 0, SDQ_INV_LOH, g.data(), ld, sg, st) == SDQ_OK);  // empty batch
    CHECK(sdq_sync(ctx) == SDQ_OK);
  }
}

}  // namespace

int main(int argc, char** argv) {
  const bool require_gpu = argc > 1 && strcmp(argv[1], "--require-gpu") == 0;
  printf("abi_check: %s\n", sdq_version());
  fflush(stdout);
  no_device_paths();
  sdq_ctx* ctx = reinterpret_cast<sdq_ctx*>(&g_checks);  // must be overwritten
  const sdq_status s = sdq_create(&ctx, 0, nullptr);
  if (s != SDQ_OK) {
    CHECK(ctx == nullptr);
    CHECK(sdq_create(&ctx, -1, nullptr) != SDQ_OK && ctx == nullptr);
    printf("abi_check: no usable device (status %d): %d checks passed without one\n", (int)s, g_checks);
    return require_gpu ? 1 : 0;
  }
  CHECK(sdq_create(nullptr, 0, nullptr) == SDQ_EINVAL);
  with_device(ctx);
  sdq_destroy(ctx);
  // a second context after the first is gone: nothing of it may linger
  CHECK(sdq_create(&ctx, 0, nullptr) == SDQ_OK);
  sdq_destroy(ctx);
  printf("abi_check: %d checks passed on device 0\n", g_checks);
  return 0;
}
