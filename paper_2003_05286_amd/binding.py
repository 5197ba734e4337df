"""Python binding of libsdq (include/sdq.h): argument marshalling only.

Every step of the method runs in the HIP library; this module turns torch
tensors into device pointers, calls the C ABI on torch's current stream and
returns torch tensors.  There is no CPU fallback: if libsdq.so is missing or
no GPU is visible the calls raise.

Instances are given as `Chain` records (one Markov chain / spin flavour):
    B_l = expk @ diag(exp(alpha * field[l-1]))      l = 1..m
with expk, expk_inv ([n, n]) and field ([m, n]) float64 CUDA tensors.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from dataclasses import dataclass

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsdq.so")

SDQ_OK, SDQ_EINVAL, SDQ_ENOMEM, SDQ_EHIP, SDQ_ERANGE, SDQ_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
SCHEME_LOH, SCHEME_PLAIN = 0, 1
STAB_QR, STAB_SVD = 0, 1

# every symbol include/sdq.h declares
EXPORTS = ("sdq_create", "sdq_destroy", "sdq_last_error", "sdq_version", "sdq_greens",
           "sdq_greens_tdisp", "sdq_logdet", "sdq_logdet_grad", "sdq_release", "sdq_udt",
           "sdq_chain_udt", "sdq_tune", "sdq_set_graphs", "sdq_set_profiling",
           "sdq_kernel_stats", "sdq_sync", "sdq_similarity", "sdq_metropolis",
           "sdq_local_sweep", "sdq_langevin", "sdq_hmc", "sdq_set_stabilizer", "sdq_greens_dense",
           "sdq_greens_tdisp_dense", "sdq_udt_complex", "sdq_kernel_names", "sdq_greens_noalloc",
           "sdq_greens_complex")


class SdqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"sdq status {status}: {msg}")
        self.status = status


class _Instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("k", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("expk", ctypes.c_void_p), ("expk_inv", ctypes.c_void_p),
                ("field", ctypes.c_void_p), ("alpha", ctypes.c_double)]


class _ComplexInstance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("k", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("slices", ctypes.c_void_p)]


class _DenseInstance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("k", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("slices", ctypes.c_void_p)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libsdq.so and declare the C signatures (works without a GPU)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_2003_05286_amd.build`")
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.sdq_create.argtypes = [P(vp), ctypes.c_int, vp]
    L.sdq_destroy.argtypes = [vp]
    L.sdq_destroy.restype = None
    L.sdq_last_error.argtypes = [vp]
    L.sdq_last_error.restype = ctypes.c_char_p
    L.sdq_version.argtypes = []
    L.sdq_version.restype = ctypes.c_char_p
    L.sdq_greens.argtypes = [vp, P(_Instance), i32, ctypes.c_int, P(vp), vp, vp, vp]
    L.sdq_greens_noalloc.argtypes = [vp, P(_Instance), i32, ctypes.c_int, P(vp), vp, vp, vp]
    L.sdq_greens_tdisp.argtypes = [vp, P(_Instance), i32, ctypes.c_int, P(i32), i32, P(vp), P(vp),
                                   vp, vp, vp]
    L.sdq_logdet.argtypes = [vp, P(_Instance), i32, vp, vp, vp, P(ctypes.c_uint64)]
    L.sdq_logdet_grad.argtypes = [vp, ctypes.c_uint64, P(_Instance), i32, P(vp), vp, vp, vp]
    L.sdq_release.argtypes = [vp, ctypes.c_uint64]
    L.sdq_udt.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    L.sdq_udt_complex.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    L.sdq_greens_complex.argtypes = [vp, P(_ComplexInstance), i32, P(vp), vp, vp, vp]
    L.sdq_chain_udt.argtypes = [vp, P(_Instance), i32, vp, vp, vp]
    L.sdq_tune.argtypes = [vp, P(i32), i32, ctypes.c_char_p]
    L.sdq_set_graphs.argtypes = [vp, ctypes.c_int]
    L.sdq_set_profiling.argtypes = [vp, ctypes.c_int]
    L.sdq_kernel_stats.argtypes = [vp, ctypes.c_char_p, P(i64), P(dbl)]
    L.sdq_kernel_names.argtypes = [vp, ctypes.c_char_p, i32]
    L.sdq_sync.argtypes = [vp]
    L.sdq_similarity.argtypes = [vp, i32, i32, vp, vp, P(vp)]
    L.sdq_metropolis.argtypes = [vp, P(_Instance), P(_Instance), i32, i32, vp, vp, vp, vp, vp, vp]
    L.sdq_local_sweep.argtypes = [vp, P(_Instance), i32, i32, vp, vp, vp]
    L.sdq_langevin.argtypes = [vp, P(_Instance), i32, i32, dbl, dbl, vp, vp, vp, vp, vp]
    L.sdq_hmc.argtypes = [vp, P(_Instance), i32, i32, dbl, i32, dbl, vp, vp, vp, vp, vp, vp, vp]
    L.sdq_set_stabilizer.argtypes = [vp, i32]
    L.sdq_greens_dense.argtypes = [vp, P(_DenseInstance), i32, P(vp), vp, vp, vp]
    L.sdq_greens_tdisp_dense.argtypes = [vp, P(_DenseInstance), i32, P(i32), i32, P(vp), P(vp), vp, vp, vp]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("sdq_destroy", "sdq_last_error", "sdq_version"):
            f.restype = ctypes.c_int
    _lib = L
    return L


def version() -> str:
    return load_library().sdq_version().decode()


@dataclass
class Chain:
    expk: torch.Tensor
    field: torch.Tensor
    alpha: float
    k: int
    expk_inv: torch.Tensor | None = None

    @property
    def n(self):
        return self.expk.shape[0]

    @property
    def m(self):
        return self.field.shape[0]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_tensor(t, name, shape, device):
    if t.dtype != torch.float64 or not t.is_contiguous() or t.device != device or tuple(t.shape) != shape:
        raise ValueError(f"{name}: need a contiguous float64 tensor of shape {shape} on {device}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


# Contexts still open when the interpreter exits are closed by an atexit
# hook, while the HIP runtime (and any profiler attached to it) is still up,
# rather than by a finalizer during teardown.
_live = weakref.WeakSet()


@atexit.register
def _close_all():
    for c in list(_live):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """An sdq context bound to one device and to torch's current stream."""

    def __init__(self, device: int | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("sdq needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = load_library()
        self.device = torch.cuda.current_device() if device is None else device
        self.tdev = torch.device("cuda", self.device)
        self.stream = torch.cuda.current_stream(self.tdev)
        h = ctypes.c_void_p()
        st = self.lib.sdq_create(ctypes.byref(h), self.device, ctypes.c_void_p(self.stream.cuda_stream))
        if st != SDQ_OK:
            raise SdqError(st, "sdq_create failed")
        self.h = h
        self._keep = []
        _live.add(self)

    def close(self):
        """Wait for the context's work and release its device memory, streams
        and graphs (sdq_destroy).  Idempotent."""
        if getattr(self, "h", None):
            self.lib.sdq_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------
    def _chk(self, st):
        if st != SDQ_OK:
            raise SdqError(st, self.lib.sdq_last_error(self.h).decode())

    def _instances(self, chains, need_inv=False):
        arr = (_Instance * max(len(chains), 1))()
        for i, c in enumerate(chains):
            n, m = c.n, c.m
            _check_tensor(c.expk, "expk", (n, n), self.tdev)
            _check_tensor(c.field, "field", (m, n), self.tdev)
            if c.expk_inv is not None:
                _check_tensor(c.expk_inv, "expk_inv", (n, n), self.tdev)
            elif need_inv:
                raise ValueError("expk_inv is required")
            arr[i] = _Instance(n, m, int(c.k), 0, c.expk.data_ptr(),
                               c.expk_inv.data_ptr() if c.expk_inv is not None else 0,
                               c.field.data_ptr(), float(c.alpha))
        return arr

    def _empty(self, *shape):
        return torch.empty(*shape, dtype=torch.float64, device=self.tdev)

    @staticmethod
    def _ptr_array(ts):
        arr = (ctypes.c_void_p * max(len(ts), 1))()
        for i, t in enumerate(ts):
            arr[i] = t.data_ptr() if t is not None else 0
        return arr

    # -- calls -------------------------------------------------------------
    def greens(self, chains, scheme=SCHEME_LOH, want_g=True):
        """Equal-time G per chain, log|det(1+B)|, sign, status."""
        cnt = len(chains)
        inst = self._instances(chains)
        gs = [self._empty(c.n, c.n) for c in chains] if want_g else [None] * cnt
        ld, sg = self._empty(cnt), self._empty(cnt)
        stt = torch.empty(cnt, dtype=torch.int32, device=self.tdev)
        self._chk(self.lib.sdq_greens(self.h, inst, cnt, scheme, self._ptr_array(gs),
                                      _ptr(ld), _ptr(sg), _ptr(stt)))
        return gs, ld, sg, stt

    def greens_noalloc(self, chains, gs, ld, sg, stt, scheme=SCHEME_LOH):
        """sdq_greens_noalloc into caller-provided outputs: gs (list of [n, n]
        float64 tensors or None), ld, sg ([count] float64), stt ([count] int32)."""
        cnt = len(chains)
        inst = self._instances(chains)
        for t, name, shape in ((ld, "logdet", (cnt,)), (sg, "sign", (cnt,))):
            _check_tensor(t, name, shape, self.tdev)
        if stt.dtype != torch.int32 or tuple(stt.shape) != (cnt,) or stt.device != self.tdev:
            raise ValueError("status: need an int32 tensor of shape [count] on the context's device")
        for c, g in zip(chains, gs):
            if g is not None:
                _check_tensor(g, "g", (c.n, c.n), self.tdev)
        self._chk(self.lib.sdq_greens_noalloc(self.h, inst, cnt, scheme, self._ptr_array(gs),
                                              _ptr(ld), _ptr(sg), _ptr(stt)))

    def greens_tdisp(self, chains, l_list, want_g=True, scheme=SCHEME_LOH):
        """G(tau_l, 0) for l in l_list ([n_l, n, n] per chain), G, logdet, sign, status."""
        cnt = len(chains)
        inst = self._instances(chains)
        ls = (ctypes.c_int32 * max(len(l_list), 1))(*[int(x) for x in l_list])
        gts = [self._empty(len(l_list), c.n, c.n) for c in chains]
        gs = [self._empty(c.n, c.n) for c in chains] if want_g else [None] * cnt
        ld, sg = self._empty(cnt), self._empty(cnt)
        stt = torch.empty(cnt, dtype=torch.int32, device=self.tdev)
        self._chk(self.lib.sdq_greens_tdisp(self.h, inst, cnt, scheme, ls, len(l_list),
                                            self._ptr_array(gts), self._ptr_array(gs),
                                            _ptr(ld), _ptr(sg), _ptr(stt)))
        return gts, gs, ld, sg, stt

    def logdet(self, chains, keep=False):
        cnt = len(chains)
        inst = self._instances(chains)
        ld, sg = self._empty(cnt), self._empty(cnt)
        stt = torch.empty(cnt, dtype=torch.int32, device=self.tdev)
        hnd = ctypes.c_uint64(0)
        self._chk(self.lib.sdq_logdet(self.h, inst, cnt, _ptr(ld), _ptr(sg), _ptr(stt),
                                      ctypes.byref(hnd) if keep else None))
        return ld, sg, stt, hnd.value

    def logdet_grad(self, chains, handle=0):
        cnt = len(chains)
        inst = self._instances(chains, need_inv=True)
        grads = [self._empty(c.m, c.n) for c in chains]
        ld, sg = self._empty(cnt), self._empty(cnt)
        stt = torch.empty(cnt, dtype=torch.int32, device=self.tdev)
        self._chk(self.lib.sdq_logdet_grad(self.h, ctypes.c_uint64(handle), inst, cnt,
                                           self._ptr_array(grads), _ptr(ld), _ptr(sg), _ptr(stt)))
        return grads, ld, sg, stt

    def release(self, handle):
        self._chk(self.lib.sdq_release(self.h, ctypes.c_uint64(handle)))

    def udt(self, w):
        """w: [count, n, n] -> U [count,n,n], D [count,n], T [count,n,n]."""
        cnt, n, _ = w.shape
        _check_tensor(w, "w", (cnt, n, n), self.tdev)
        u, t, d = self._empty(cnt, n, n), self._empty(cnt, n, n), self._empty(cnt, n)
        self._chk(self.lib.sdq_udt(self.h, n, cnt, _ptr(w), _ptr(u), _ptr(d), _ptr(t)))
        return u, d, t

    def udt_complex(self, w):
        """w: complex128 [count, n, n] -> U [count,n,n] complex, D [count,n] real,
        T [count,n,n] complex (sdq_udt_complex)."""
        if w.dim() != 3 or w.shape[1] != w.shape[2]:
            raise ValueError(f"w: need shape [count, n, n], got {tuple(w.shape)}")
        cnt, n, _ = w.shape
        if w.dtype != torch.complex128 or not w.is_contiguous() or w.device != self.tdev:
            raise ValueError(f"w: need a contiguous complex128 tensor on {self.tdev}, got {w.dtype} on {w.device}")
        u = torch.empty(cnt, n, n, dtype=torch.complex128, device=self.tdev)
        t = torch.empty(cnt, n, n, dtype=torch.complex128, device=self.tdev)
        d = self._empty(cnt, n)
        self._chk(self.lib.sdq_udt_complex(self.h, n, cnt, _ptr(torch.view_as_real(w)),
                                           _ptr(torch.view_as_real(u)), _ptr(d), _ptr(torch.view_as_real(t))))
        return u, d, t

    def greens_complex(self, slices, k):
        """Chains of complex slices (sdq_greens_complex).  slices: list of
        complex128 tensors [m, n, n] (one per chain, B_l = slices[l-1]).
        Returns (G list of complex [n, n], logdet [count], phase complex
        [count], status [count] int32)."""
        cnt = len(slices)
        arr = (_ComplexInstance * max(cnt, 1))()
        ks = k if isinstance(k, (list, tuple)) else [k] * cnt
        gs = []
        for i, sl in enumerate(slices):
            if (sl.dim() != 3 or sl.shape[1] != sl.shape[2] or sl.dtype != torch.complex128
                    or not sl.is_contiguous() or sl.device != self.tdev):
                raise ValueError(f"slices[{i}]: need a contiguous complex128 [m, n, n] tensor on {self.tdev}")
            m, n = sl.shape[0], sl.shape[1]
            arr[i] = _ComplexInstance(n, m, int(ks[i]), 0, sl.data_ptr())
            gs.append(torch.empty(n, n, dtype=torch.complex128, device=self.tdev))
        ld = self._empty(cnt)
        ph = self._empty(cnt, 2)
        stt = torch.empty(cnt, dtype=torch.int32, device=self.tdev)
        self._chk(self.lib.sdq_greens_complex(self.h, arr, cnt, self._ptr_array(gs), _ptr(ld), _ptr(ph),
                                              _ptr(stt)))
        return gs, ld, torch.view_as_complex(ph), stt

    def chain_udt(self, chains):
        cnt = len(chains)
        n = chains[0].n
        inst = self._instances(chains)
        u, t, d = self._empty(cnt, n, n), self._empty(cnt, n, n), self._empty(cnt, n)
        self._chk(self.lib.sdq_chain_udt(self.h, inst, cnt, _ptr(u), _ptr(d), _ptr(t)))
        return u, d, t

    def metropolis(self, cur, prop, nf, dS, u, logdet, sign):
        """One global-update Metropolis step (sdq_metropolis).  cur / prop:
        lists of Chain, count * nf entries, flavour f of chain c at c * nf + f;
        dS, u: device [count]; logdet, sign: device [count * nf], the current
        fields' values, updated in place.  Returns (accept [count] int32,
        status [count * nf] int32)."""
        total = len(cur)
        if len(prop) != total or nf < 1 or total % nf:
            raise ValueError("cur and prop need count * nf entries each")
        count = total // nf
        for t, name, shape in ((dS, "dS", (count,)), (u, "u", (count,)), (logdet, "logdet", (total,)),
                               (sign, "sign", (total,))):
            _check_tensor(t, name, shape, self.tdev)
        ci, pi = self._instances(cur), self._instances(prop)
        acc = torch.empty(count, dtype=torch.int32, device=self.tdev)
        st = torch.empty(total, dtype=torch.int32, device=self.tdev)
        self._chk(self.lib.sdq_metropolis(self.h, ci, pi, count, nf, _ptr(dS), _ptr(u), _ptr(logdet),
                                          _ptr(sign), _ptr(acc), _ptr(st)))
        return acc, st

    def _dense(self, slices, k):
        arr = (_DenseInstance * max(len(slices), 1))()
        for i, t in enumerate(slices):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.tdev or t.dim() != 3 \
                    or t.shape[1] != t.shape[2]:
                raise ValueError(f"slices[{i}]: need a contiguous float64 [m, n, n] tensor on {self.tdev}")
            arr[i] = _DenseInstance(t.shape[2], t.shape[0], int(k), 0, t.data_ptr())
        return arr

    def greens_dense(self, slices, k):
        """Equal-time G, log|det(1+B)|, sign and status for chains of dense
        slices (sdq_greens_dense): slices is a list of device [m, n, n]
        float64 tensors, B_l = slices[c][l-1]."""
        cnt = len(slices)
        arr = self._dense(slices, k)
        gs = [self._empty(t.shape[2], t.shape[2]) for t in slices]
        ld, sg = self._empty(cnt), self._empty(cnt)
        st = torch.empty(cnt, dtype=torch.int32, device=self.tdev)
        self._chk(self.lib.sdq_greens_dense(self.h, arr, cnt, self._ptr_array(gs), _ptr(ld), _ptr(sg), _ptr(st)))
        return gs, ld, sg, st

    def greens_tdisp_dense(self, slices, k, l_list):
        """G(tau_l, 0) ([n_l, n, n] per chain), G, log|det|, sign, status for
        chains of dense slices (sdq_greens_tdisp_dense); l ascending in
        [0, m]."""
        cnt = len(slices)
        arr = self._dense(slices, k)
        ls = (ctypes.c_int32 * max(len(l_list), 1))(*[int(x) for x in l_list])
        gts = [self._empty(len(l_list), t.shape[2], t.shape[2]) for t in slices]
        gs = [self._empty(t.shape[2], t.shape[2]) for t in slices]
        ld, sg = self._empty(cnt), self._empty(cnt)
        st = torch.empty(cnt, dtype=torch.int32, device=self.tdev)
        self._chk(self.lib.sdq_greens_tdisp_dense(self.h, arr, cnt, ls, len(l_list), self._ptr_array(gts),
                                                  self._ptr_array(gs), _ptr(ld), _ptr(sg), _ptr(st)))
        return gts, gs, ld, sg, st

    def set_stabilizer(self, stab):
        """STAB_QR (default) or STAB_SVD for every later sweep (sdq_set_stabilizer)."""
        self._chk(self.lib.sdq_set_stabilizer(self.h, int(stab)))

    def langevin(self, chains, nf, eps, inv_var, noise, force=True):
        """One Langevin step (sdq_langevin): chains = count * nf Chains
        (flavours of a chain consecutive, sharing its field tensor, which is
        updated in place); noise: device [count, m, n] standard normals.
        Returns (force [count, m, n] or None, logdet [count * nf], sign
        [count * nf], status [count * nf] int32), logdet and sign of the
        field before the step."""
        total = len(chains)
        if nf < 1 or total % nf:
            raise ValueError("chains must hold count * nf entries")
        count = total // nf
        c0 = chains[0]
        _check_tensor(noise, "noise", (count, c0.m, c0.n), self.tdev)
        inst = self._instances(chains, need_inv=True)
        frc = torch.empty(count, c0.m, c0.n, dtype=torch.float64, device=self.tdev) if force else None
        ld, sg = self._empty(total), self._empty(total)
        st = torch.empty(total, dtype=torch.int32, device=self.tdev)
        self._chk(self.lib.sdq_langevin(self.h, inst, count, nf, float(eps), float(inv_var), _ptr(noise),
                                        _ptr(frc) if frc is not None else None, _ptr(ld), _ptr(sg),
                                        _ptr(st)))
        return frc, ld, sg, st

    def hmc(self, chains, nf, eps, nsteps, inv_var, mom, u):
        """One hybrid Monte Carlo trajectory per chain (sdq_hmc): chains =
        count * nf Chains (flavours of a chain consecutive, sharing its field
        tensor, updated in place); mom: device [count, m, n] standard normals;
        u: device [count] uniforms.  Returns (accept [count] int32, dH
        [count], logdet [count * nf], sign [count * nf], status [count * nf]
        int32), logdet and sign of the field the chain ends on."""
        total = len(chains)
        if nf < 1 or total % nf:
            raise ValueError("chains must hold count * nf entries")
        count = total // nf
        c0 = chains[0]
        _check_tensor(mom, "mom", (count, c0.m, c0.n), self.tdev)
        _check_tensor(u, "u", (count,), self.tdev)
        inst = self._instances(chains, need_inv=True)
        acc = torch.empty(count, dtype=torch.int32, device=self.tdev)
        dh = self._empty(count)
        ld, sg = self._empty(total), self._empty(total)
        st = torch.empty(total, dtype=torch.int32, device=self.tdev)
        self._chk(self.lib.sdq_hmc(self.h, inst, count, nf, float(eps), int(nsteps), float(inv_var), _ptr(mom),
                                   _ptr(u), _ptr(ld), _ptr(sg), _ptr(acc), _ptr(dh), _ptr(st)))
        return acc, dh, ld, sg, st

    def local_sweep(self, chains, nf, unif):
        """One sweep of local updates (sdq_local_sweep): chains = count * nf
        Chains (flavours of a chain consecutive, sharing its field tensor,
        which is updated in place); unif: device [count, m, n].  Returns
        (accepted [count] int32, status [count * nf] int32)."""
        total = len(chains)
        if nf < 1 or total % nf:
            raise ValueError("chains must hold count * nf entries")
        count = total // nf
        c0 = chains[0]
        _check_tensor(unif, "unif", (count, c0.m, c0.n), self.tdev)
        inst = self._instances(chains, need_inv=True)
        acc = torch.empty(count, dtype=torch.int32, device=self.tdev)
        st = torch.empty(total, dtype=torch.int32, device=self.tdev)
        self._chk(self.lib.sdq_local_sweep(self.h, inst, count, nf, _ptr(unif), _ptr(acc), _ptr(st)))
        return acc, st

    def similarity(self, mats, left, right):
        """M <- left @ M @ right in place for every n x n matrix of `mats` (a
        list of device tensors whose last two dims are n x n; every matrix of
        each is transformed).  With left = E^{-1/2}, right = E^{1/2} this maps
        G and G(tau,0) of the slices E diag(v) to those of the symmetric
        slices E^{1/2} diag(v) E^{1/2}."""
        n = left.shape[0]
        _check_tensor(left, "left", (n, n), self.tdev)
        _check_tensor(right, "right", (n, n), self.tdev)
        ptrs = []
        for t in mats:
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device != self.tdev or \
                    t.dim() < 2 or tuple(t.shape[-2:]) != (n, n):
                raise ValueError(f"mats: need contiguous float64 (..., {n}, {n}) tensors on {self.tdev}")
            for b in range(t.numel() // (n * n)):
                ptrs.append(t.data_ptr() + b * n * n * 8)
        arr = (ctypes.c_void_p * max(len(ptrs), 1))(*ptrs)
        self._chk(self.lib.sdq_similarity(self.h, n, len(ptrs), _ptr(left), _ptr(right), arr))

    def tune(self, n_list, cache_path=None):
        arr = (ctypes.c_int32 * len(n_list))(*n_list)
        self._chk(self.lib.sdq_tune(self.h, arr, len(n_list),
                                    cache_path.encode() if cache_path else None))

    def set_graphs(self, enable: bool):
        self._chk(self.lib.sdq_set_graphs(self.h, int(enable)))

    def set_profiling(self, enable: bool):
        self._chk(self.lib.sdq_set_profiling(self.h, int(enable)))

    def kernel_stats(self, name):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0)
        self._chk(self.lib.sdq_kernel_stats(self.h, name.encode(), ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def kernel_names(self):
        buf = ctypes.create_string_buffer(1 << 16)
        self._chk(self.lib.sdq_kernel_names(self.h, buf, len(buf)))
        return [x for x in buf.value.decode().split(",") if x]

    def sync(self):
        self._chk(self.lib.sdq_sync(self.h))


_default = {}


def context(device: int | None = None) -> Context:
    dev = torch.cuda.current_device() if device is None else device
    key = (dev, torch.cuda.current_stream(dev).cuda_stream)
    if key not in _default:
        _default[key] = Context(dev)
    return _default[key]


class LogDet1pB(torch.autograd.Function):
    """log|det(1 + B_m ... B_1)| of a batch of chains with a hand-written
    adjoint: d/d field[l-1, i] = alpha (1 - G_l)_ii (see sdq_logdet_grad).

    forward(field [count, m, n], expk [n, n], expk_inv [n, n], alpha, k)
      -> (logdet [count], sign [count]); the sign carries no gradient."""

    @staticmethod
    def forward(ctx, field, expk, expk_inv, alpha, k):
        c = context(field.device.index)
        chains = [Chain(expk, field[i], alpha, k, expk_inv) for i in range(field.shape[0])]
        # keep the forward stages for the backward only when one will follow
        ld, sg, stt, hnd = c.logdet(chains, keep=bool(ctx.needs_input_grad[0]))
        ctx.handle = hnd
        ctx.sdq = c
        ctx.args = (expk, expk_inv, alpha, k)
        ctx.save_for_backward(field)
        ctx.mark_non_differentiable(sg)
        return ld, sg

    @staticmethod
    def backward(ctx, g_ld, g_sg):
        (field,) = ctx.saved_tensors
        expk, expk_inv, alpha, k = ctx.args
        c = ctx.sdq
        chains = [Chain(expk, field[i], alpha, k, expk_inv) for i in range(field.shape[0])]
        if ctx.handle:
            # first backward: reuse the forward stages, then free them
            try:
                grads, _, _, _ = c.logdet_grad(chains, handle=ctx.handle)
            finally:
                c.release(ctx.handle)
                ctx.handle = 0
        else:
            # a repeated backward (retain_graph) recomputes the forward stages
            grads, _, _, _ = c.logdet_grad(chains)
        grad = torch.stack(grads) * g_ld.view(-1, 1, 1)
        return grad, None, None, None, None
