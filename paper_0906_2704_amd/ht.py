"""Thin Python binding of libht (include/ht.h): argument marshalling only.

Every function takes torch tensors that live on the current HIP device and passes their
data pointers and the current torch stream to the C ABI; all arithmetic happens in the
library's kernels.  There is no fallback: if libht.so is missing or a call fails, a
RuntimeError is raised.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libht.so")

HT_FAMILY_PAPER, HT_FAMILY_DST = 0, 1
HT_NORM_IDENTITY, HT_NORM_SECOND_DIFF = 0, 1
KIND_NAMES = {1: "AR", 2: "C", 3: "F", 4: "DST2", 5: "DST3", 6: "P", 7: "R", 8: "F3"}
NORMS = {"I": HT_NORM_IDENTITY, "D2": HT_NORM_SECOND_DIFF}
FAMILIES = {"paper": HT_FAMILY_PAPER, "dst": HT_FAMILY_DST, "paper+dst3": 2, "periodic": 3, "reflective": 4}
PRECISIONS = {"f64": 0, "bf16x3": 1, "f16x3": 2, "f32": 3}
SPECTRUM_FACTORS, SPECTRUM_FULL = 0, 1

_lib = None


class HTError(RuntimeError):
    pass


def lib():
    """Load libht.so (built in-tree by paper_0906_2704_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise HTError("libht.so is not built (run __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    P, I64, I32, VP = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    L.ht_plan_create.argtypes = [ctypes.c_int, ctypes.POINTER(I64), ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, I64, ctypes.POINTER(P)]
    L.ht_plan_destroy.argtypes = [P]
    L.ht_plan_kind.argtypes = [P, ctypes.c_int]
    L.ht_plan_is_complex.argtypes = [P]
    L.ht_eigs.argtypes = [P, VP, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.c_int, VP, VP, I64, VP]
    L.ht_transform_inv.argtypes = [P, VP, VP, I64, VP]
    L.ht_transform_fwd.argtypes = [P, VP, VP, I64, VP]
    L.ht_eigs2d.argtypes = [P, VP, I64, I64, I64, I64, ctypes.c_int, VP, VP, I64, VP]
    L.ht_tikhonov_filter.argtypes = [P, VP, VP, VP, I64, ctypes.c_int, VP, VP, I64, VP]
    L.ht_gcv_scan.argtypes = [P, VP, VP, VP, I64, ctypes.c_int, VP, I32, ctypes.c_int, VP, VP, VP, I64, VP]
    L.ht_gcv_scan_exact.argtypes = [P, VP, VP, VP, I64, ctypes.c_int, VP, I32, ctypes.c_int, VP, VP, VP, I64, VP]
    L.ht_gcv_scan_exact_static.argtypes = [P, VP, VP, VP, I64, ctypes.c_int, VP, I32, ctypes.c_int, VP, VP, VP, I64,
                                           VP]
    L.ht_plan_set_precision.argtypes = [P, ctypes.c_int]
    L.ht_plan_reserve_exact_gcv.argtypes = [P, I32]
    L.ht_plan_precision.argtypes = [P]
    L.ht_status_str.argtypes = [ctypes.c_int]
    L.ht_status_str.restype = ctypes.c_char_p
    L.ht_last_error.restype = ctypes.c_char_p
    for name in ("ht_plan_create", "ht_plan_destroy", "ht_eigs", "ht_eigs2d", "ht_transform_inv", "ht_transform_fwd",
                 "ht_tikhonov_filter", "ht_gcv_scan", "ht_gcv_scan_exact", "ht_plan_set_precision", "ht_plan_precision",
                 "ht_plan_reserve_exact_gcv", "ht_gcv_scan_exact_static"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status, what):
    if status != 0:
        L = lib()
        raise HTError("%s failed: %s (%s)" % (what, L.ht_status_str(status).decode(),
                                               L.ht_last_error().decode()))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype, name):
    if t is None:
        return None
    if not t.is_cuda:
        raise HTError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise HTError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise HTError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """A transform plan (ht_plan_create).  `n` is an int (1D) or a pair (2D)."""

    def __init__(self, n, degree, psf_symmetric=True, family="paper", max_batch=1):
        L = lib()
        dims = [int(n)] if isinstance(n, int) else [int(v) for v in n]
        self.ndim = len(dims)
        self.n = dims
        arr = (ctypes.c_int64 * self.ndim)(*dims)
        h = ctypes.c_void_p()
        _check(L.ht_plan_create(self.ndim, arr, int(degree), int(bool(psf_symmetric)),
                                FAMILIES.get(family, family), int(max_batch), ctypes.byref(h)),
               "ht_plan_create")
        self._h = h
        self.degree = degree
        self.max_batch = max_batch
        self.kinds = [KIND_NAMES[L.ht_plan_kind(h, a)] for a in range(self.ndim)]
        self.is_complex = bool(L.ht_plan_is_complex(h))
        self.coeff_dtype = torch.complex128 if self.is_complex else torch.float64

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            lib().ht_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_precision(self, precision):
        """Core arithmetic: "f64" (default), "bf16x3" or "f16x3" (ht_plan_set_precision)."""
        _check(lib().ht_plan_set_precision(self._h, PRECISIONS.get(precision, precision)), "ht_plan_set_precision")

    def reserve_exact_gcv(self, max_k):
        """Size the 2D exact GCV workspace for grids of up to max_k values (set-up call)."""
        _check(lib().ht_plan_reserve_exact_gcv(self._h, int(max_k)), "ht_plan_reserve_exact_gcv")

    @property
    def precision(self):
        code = lib().ht_plan_precision(self._h)
        return {v: k for k, v in PRECISIONS.items()}[code]

    def item_shape(self):
        return tuple(self.n)

    def spectrum_len(self):
        return sum(self.n) if self.ndim == 2 else self.n[0]


def ht_eigs(plan, psf, psf_len, psf_center, norm, batch=1, d=None, s=None):
    """Eigenvalues d and s (see include/ht.h).  psf: float64 device tensor."""
    L = lib()
    m = plan.spectrum_len()
    if d is None:
        d = torch.empty((batch, m), dtype=plan.coeff_dtype, device=psf.device)
    if s is None:
        s = torch.empty((batch, m), dtype=torch.float64, device=psf.device)
    lens = (ctypes.c_int64 * plan.ndim)(*[int(v) for v in psf_len])
    cens = (ctypes.c_int64 * plan.ndim)(*[int(v) for v in psf_center])
    _check(L.ht_eigs(plan.handle, _ptr(psf, torch.float64, "psf"), lens, cens, NORMS.get(norm, norm),
                     _ptr(d, plan.coeff_dtype, "d"), _ptr(s, torch.float64, "s"), int(batch), _stream()),
           "ht_eigs")
    return d, s


def ht_eigs2d(plan, psf, psf_center, norm, d=None, s=None):
    """Eigenvalues for general 2D masks (see include/ht.h): psf float64 device tensor
    [batch, len0, len1] or [len0, len1]; returns d, s of shape [batch, n0, n1]."""
    L = lib()
    if plan.ndim != 2:
        raise ValueError("ht_eigs2d needs a 2D plan")
    H = psf if psf.dim() == 3 else psf.unsqueeze(0)
    batch, len0, len1 = H.shape
    n0, n1 = plan.n
    if d is None:
        d = torch.empty((batch, n0, n1), dtype=plan.coeff_dtype, device=psf.device)
    if s is None:
        s = torch.empty((batch, n0, n1), dtype=torch.float64, device=psf.device)
    _check(L.ht_eigs2d(plan.handle, _ptr(H, torch.float64, "psf"), int(len0), int(len1), int(psf_center[0]),
                       int(psf_center[1]), NORMS.get(norm, norm), _ptr(d, plan.coeff_dtype, "d"),
                       _ptr(s, torch.float64, "s"), int(batch), _stream()), "ht_eigs2d")
    return d, s


def _spectrum(plan, d):
    """(eig_batch, layout) of a spectrum tensor: 2D plans take the factors of ht_eigs
    (n0 + n1 entries) or the full [eig_batch, n0, n1] arrays of ht_eigs2d."""
    if plan.ndim == 2:
        img = _item(plan)
        if d.numel() == plan.spectrum_len():
            return 1, SPECTRUM_FACTORS
        if d.numel() % img == 0:
            return d.numel() // img, SPECTRUM_FULL
        raise ValueError("spectrum of %d entries fits neither layout" % d.numel())
    return d.numel() // plan.spectrum_len(), SPECTRUM_FULL


def ht_transform_inv(plan, signal, out=None):
    L = lib()
    batch = signal.numel() // _item(plan)
    if out is None:
        out = torch.empty(signal.shape, dtype=plan.coeff_dtype, device=signal.device)
    _check(L.ht_transform_inv(plan.handle, _ptr(signal, torch.float64, "signal"),
                              _ptr(out, plan.coeff_dtype, "coeff"), batch, _stream()), "ht_transform_inv")
    return out


def ht_transform_fwd(plan, coeff, out=None):
    L = lib()
    batch = coeff.numel() // _item(plan)
    if out is None:
        out = torch.empty(coeff.shape, dtype=torch.float64, device=coeff.device)
    _check(L.ht_transform_fwd(plan.handle, _ptr(coeff, plan.coeff_dtype, "coeff"),
                              _ptr(out, torch.float64, "signal"), batch, _stream()), "ht_transform_fwd")
    return out


def ht_tikhonov_filter(plan, coeff, d, s, mu, out=None):
    L = lib()
    batch = coeff.numel() // _item(plan)
    eig_batch, layout = _spectrum(plan, d)
    if out is None:
        out = torch.empty_like(coeff)
    _check(L.ht_tikhonov_filter(plan.handle, _ptr(coeff, plan.coeff_dtype, "coeff"),
                                _ptr(d, plan.coeff_dtype, "d"), _ptr(s, torch.float64, "s"), eig_batch, layout,
                                _ptr(mu, torch.float64, "mu"), _ptr(out, plan.coeff_dtype, "fhat"),
                                batch, _stream()), "ht_tikhonov_filter")
    return out


def ht_gcv_scan(plan, coeff, d, s, mu_grid, want_G=True, G=None, kb=None, mb=None):
    """Returns (G or None, k_best int32 [batch], mu_best float64 [batch])."""
    L = lib()
    batch = coeff.numel() // _item(plan)
    eig_batch, layout = _spectrum(plan, d)
    K = mu_grid.shape[-1]
    per_item = 1 if mu_grid.dim() == 2 else 0
    dev = coeff.device
    if G is None and want_G:
        G = torch.empty((batch, K), dtype=torch.float64, device=dev)
    if kb is None:
        kb = torch.empty(batch, dtype=torch.int32, device=dev)
    if mb is None:
        mb = torch.empty(batch, dtype=torch.float64, device=dev)
    _check(L.ht_gcv_scan(plan.handle, _ptr(coeff, plan.coeff_dtype, "coeff"), _ptr(d, plan.coeff_dtype, "d"),
                         _ptr(s, torch.float64, "s"), eig_batch, layout, _ptr(mu_grid, torch.float64, "mu_grid"),
                         int(K), per_item, _ptr(G, torch.float64, "G"), _ptr(kb, torch.int32, "k_best"),
                         _ptr(mb, torch.float64, "mu_best"), batch, _stream()), "ht_gcv_scan")
    return G, kb, mb


def ht_gcv_scan_exact(plan, coeff, d, s, mu_grid, want_G=True, G=None, kb=None, mb=None):
    """Eq. gcv (exact residual norm); returns (G or None, k_best, mu_best)."""
    L = lib()
    batch = coeff.numel() // _item(plan)
    eig_batch, layout = _spectrum(plan, d)
    K = mu_grid.shape[-1]
    per_item = 1 if mu_grid.dim() == 2 else 0
    dev = coeff.device
    if G is None and want_G:
        G = torch.empty((batch, K), dtype=torch.float64, device=dev)
    if kb is None:
        kb = torch.empty(batch, dtype=torch.int32, device=dev)
    if mb is None:
        mb = torch.empty(batch, dtype=torch.float64, device=dev)
    _check(L.ht_gcv_scan_exact(plan.handle, _ptr(coeff, plan.coeff_dtype, "coeff"), _ptr(d, plan.coeff_dtype, "d"),
                               _ptr(s, torch.float64, "s"), eig_batch, layout, _ptr(mu_grid, torch.float64, "mu_grid"),
                               int(K), per_item, _ptr(G, torch.float64, "G"), _ptr(kb, torch.int32, "k_best"),
                               _ptr(mb, torch.float64, "mu_best"), batch, _stream()), "ht_gcv_scan_exact")
    return G, kb, mb


def _item(plan):
    out = 1
    for v in plan.n:
        out *= v
    return out


def _batch_sigs(L):
    P, I64, I32, VP = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    L.ht_batch_create.argtypes = [I64, VP, VP, VP, ctypes.c_int, VP, VP, ctypes.POINTER(P)]
    L.ht_batch_create.restype = ctypes.c_int
    L.ht_batch_destroy.argtypes = [P]
    L.ht_batch_destroy.restype = ctypes.c_int
    L.ht_batch_total_length.argtypes = [P]
    L.ht_batch_total_length.restype = I64
    L.ht_batch_psf_total.argtypes = [P]
    L.ht_batch_psf_total.restype = I64
    L.ht_batch_restore.argtypes = [P, VP, VP, ctypes.c_int, VP, I32, VP, VP, VP, VP, VP]
    L.ht_batch_restore.restype = ctypes.c_int
    L.ht_batch_schedule.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int)]
    L.ht_batch_schedule.restype = ctypes.c_int
    L.ht_batch_class_mask.argtypes = [P, ctypes.c_uint]
    L.ht_batch_class_mask.restype = ctypes.c_int
    L.ht_batch_class_count.argtypes = [P, ctypes.c_int]
    L.ht_batch_class_count.restype = ctypes.c_int


NCLASS = 6


class Batch:
    """A ragged batch (ht_batch_create).  All arguments are host sequences of length count."""

    def __init__(self, n, degree, psf_len, psf_center, psf_symmetric=None, family="paper+dst3"):
        import numpy as np
        L = lib()
        if not hasattr(L, "_batch_ready"):
            _batch_sigs(L)
            L._batch_ready = True
        count = len(n)
        self.count = count
        self.n = np.asarray(n, dtype=np.int64)
        self._keep = [np.ascontiguousarray(n, dtype=np.int64), np.ascontiguousarray(degree, dtype=np.int32),
                      np.ascontiguousarray(np.ones(count) if psf_symmetric is None else psf_symmetric,
                                           dtype=np.int32),
                      np.ascontiguousarray(psf_len, dtype=np.int64), np.ascontiguousarray(psf_center, dtype=np.int64)]
        h = ctypes.c_void_p()
        k = self._keep
        _check(L.ht_batch_create(count, k[0].ctypes.data, k[1].ctypes.data, k[2].ctypes.data,
                                 FAMILIES.get(family, family), k[3].ctypes.data, k[4].ctypes.data, ctypes.byref(h)),
               "ht_batch_create")
        self._h = h
        self.total_length = int(L.ht_batch_total_length(h))
        self.psf_total = int(L.ht_batch_psf_total(h))
        self.offsets = np.concatenate([[0], np.cumsum(self.n)]).astype(np.int64)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            lib().ht_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def schedule(self, size_class, workgroups=0, variant=-1):
        """Set / query (workgroups, variant) of a size class; returns the values in effect."""
        cur, var = ctypes.c_int(), ctypes.c_int()
        _check(lib().ht_batch_schedule(self._h, int(size_class), int(workgroups), int(variant), ctypes.byref(cur),
                                       ctypes.byref(var)), "ht_batch_schedule")
        return cur.value, var.value

    def class_mask(self, mask):
        _check(lib().ht_batch_class_mask(self._h, int(mask)), "ht_batch_class_mask")

    def class_count(self, size_class):
        return int(lib().ht_batch_class_count(self._h, int(size_class)))


def ht_batch_restore(batch, signal, psf, norm, mu_grid, restored=None, G=None, kb=None, mb=None, want_G=True):
    """Returns (restored, G or None, k_best, mu_best)."""
    L = lib()
    dev = signal.device
    K = mu_grid.shape[-1]
    if restored is None:
        restored = torch.empty(batch.total_length, dtype=torch.float64, device=dev)
    if G is None and want_G:
        G = torch.empty((batch.count, K), dtype=torch.float64, device=dev)
    if kb is None:
        kb = torch.empty(batch.count, dtype=torch.int32, device=dev)
    if mb is None:
        mb = torch.empty(batch.count, dtype=torch.float64, device=dev)
    if signal.numel() != batch.total_length or psf.numel() != batch.psf_total or mu_grid.numel() != batch.count * K:
        raise HTError("ht_batch_restore: array sizes do not match the batch")
    _check(L.ht_batch_restore(batch.handle, _ptr(signal, torch.float64, "signal"), _ptr(psf, torch.float64, "psf"),
                              NORMS.get(norm, norm), _ptr(mu_grid, torch.float64, "mu_grid"), int(K),
                              _ptr(restored, torch.float64, "restored"), _ptr(G, torch.float64, "G"),
                              _ptr(kb, torch.int32, "k_best"), _ptr(mb, torch.float64, "mu_best"), _stream()),
           "ht_batch_restore")
    return restored, G, kb, mb


# ----------------------------------------------------------------------------- learned mu

def _learned_sigs(L):
    I64, I32, VP, F = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_float
    Ci = ctypes.c_int
    L.ht_batch_features.argtypes = [VP, VP, VP, VP, VP, VP, VP]
    L.ht_batch_restore_learned.argtypes = [VP, VP, VP, VP, Ci, VP, I32, VP, I32, VP, VP, VP, VP, VP]
    L.ht_batch_restore_fused.argtypes = [VP, VP, VP, Ci, VP, I32, ctypes.POINTER(MlpWeights), I32, VP, VP, VP, VP, VP,
                                         VP, VP]
    L.ht_gemm_bf16.argtypes = [Ci, Ci, Ci, VP, I64, I64, VP, I64, I64, VP, Ci, VP, VP, I64, VP, VP]
    L.ht_to_bf16.argtypes = [VP, VP, I64, Ci, VP, VP, VP]
    L.ht_from_bf16.argtypes = [VP, VP, I64, VP]
    L.ht_gelu_backward.argtypes = [VP, VP, VP, VP, I64, VP]
    L.ht_colsum.argtypes = [VP, I64, Ci, VP, VP, VP]
    L.ht_mse_grad.argtypes = [VP, VP, VP, VP, I64, VP]
    L.ht_outer.argtypes = [VP, VP, VP, I64, Ci, VP]
    L.ht_adam.argtypes = [VP, VP, VP, VP, I64, F, F, F, F, I64, VP, VP]
    L.ht_transpose_bf16.argtypes = [VP, VP, Ci, Ci, VP]
    L.ht_mlp_param_count.argtypes = []
    L.ht_mlp_param_count.restype = I64
    L.ht_mlp_create.argtypes = [I64, ctypes.POINTER(VP)]
    L.ht_mlp_destroy.argtypes = [VP]
    L.ht_mlp_set_params.argtypes = [VP, VP, VP]
    L.ht_mlp_get.argtypes = [VP, Ci, VP, VP]
    L.ht_mlp_set_state.argtypes = [VP, VP, VP, I64, VP, VP, VP]
    L.ht_mlp_steps.argtypes = [VP]
    L.ht_mlp_steps.restype = I64
    L.ht_mlp_fit_standardisation.argtypes = [VP, VP, I64, VP]
    L.ht_mlp_forward.argtypes = [VP, VP, I64, VP, VP]
    L.ht_mlp_backward.argtypes = [VP, VP, I64, VP, VP]
    L.ht_mlp_predict.argtypes = [VP, VP, I64, VP, VP]
    L.ht_mlp_adam_step.argtypes = [VP, F, VP]
    L.ht_mlp_train_step.argtypes = [VP, VP, VP, VP, I64, F, VP, VP]
    L.ht_mlp_weights_of.argtypes = [VP, ctypes.POINTER(MlpWeights)]
    L.ht_log10_labels.argtypes = [VP, VP, I64, VP]
    L.ht_lambda_predict.argtypes = [VP, VP, VP, VP, VP, VP, VP, VP, VP]
    L.ht_batch_count.argtypes = [VP]
    L.ht_batch_count.restype = I64
    for name in ("ht_batch_features", "ht_batch_restore_learned", "ht_batch_restore_fused", "ht_gemm_bf16", "ht_to_bf16", "ht_from_bf16",
                 "ht_gelu_backward", "ht_colsum", "ht_mse_grad", "ht_outer", "ht_adam", "ht_transpose_bf16", "ht_mlp_create",
                 "ht_mlp_destroy", "ht_mlp_set_params", "ht_mlp_get", "ht_mlp_set_state", "ht_mlp_fit_standardisation",
                 "ht_mlp_forward", "ht_mlp_predict", "ht_mlp_backward", "ht_mlp_adam_step", "ht_mlp_train_step", "ht_mlp_weights_of",
                 "ht_log10_labels", "ht_lambda_predict"):
        getattr(L, name).restype = ctypes.c_int


def _llib():
    L = lib()
    if not hasattr(L, "_learned_ready"):
        _learned_sigs(L)
        L._learned_ready = True
    return L


def _p(t, name, dtype=None):
    if t is None:
        return None
    if dtype is not None and t.dtype != dtype:
        raise HTError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_cuda or not t.is_contiguous():
        raise HTError("%s must be a contiguous device tensor" % name)
    return ctypes.c_void_p(t.data_ptr())


BF16 = torch.bfloat16


class MlpWeights(ctypes.Structure):
    """ht_mlp_weights: device pointers of the network (bfloat16 weights [in][out], float32
    biases, feature standardisation)."""
    _fields_ = [("w", ctypes.c_void_p * 4), ("b", ctypes.c_void_p * 4), ("mean", ctypes.c_void_p),
                ("std", ctypes.c_void_p)]


def mlp_weights(wb, biases, mean, std):
    """MlpWeights from four bfloat16 weight tensors, four float32 bias tensors, mean, std."""
    m = MlpWeights()
    for l in range(4):
        m.w[l] = _p(wb[l], "w%d" % l, torch.bfloat16).value
        m.b[l] = _p(biases[l], "b%d" % l, torch.float32).value
    m.mean = _p(mean, "mean", torch.float32).value
    m.std = _p(std, "std", torch.float32).value
    return m


def ht_batch_restore_fused(batch, signal, psf, norm, mu_grid, net, cert_half=8, restored=None, kb=None, mb=None,
                           fallback=None, pred=None, features=None):
    """One-pass learned-mu restoration (features, network, certificate, filter, forward).
    `net` is an MlpWeights.  Returns (restored, k_best, mu_best, fallback, pred)."""
    L = _llib()
    dev = signal.device
    K = mu_grid.shape[-1]
    restored = torch.empty_like(signal) if restored is None else restored
    kb = torch.empty(batch.count, dtype=torch.int32, device=dev) if kb is None else kb
    mb = torch.empty(batch.count, dtype=torch.float64, device=dev) if mb is None else mb
    fallback = torch.empty(batch.count, dtype=torch.int32, device=dev) if fallback is None else fallback
    pred = torch.empty(batch.count, dtype=torch.float32, device=dev) if pred is None else pred
    _check(L.ht_batch_restore_fused(batch.handle, _p(signal, "signal", torch.float64), _p(psf, "psf", torch.float64),
                                    NORMS.get(norm, norm), _p(mu_grid, "mu_grid", torch.float64), int(K),
                                    ctypes.byref(net), int(cert_half), _p(restored, "restored", torch.float64),
                                    _p(kb, "k_best", torch.int32), _p(mb, "mu_best", torch.float64),
                                    _p(fallback, "fallback", torch.int32), _p(pred, "pred", torch.float32),
                                    _p(features, "features", torch.float32), _stream()), "ht_batch_restore_fused")
    return restored, kb, mb, fallback, pred


def ht_batch_features(batch, signal, psf, coeff=None, features=None, spectrum=None):
    """Returns (coeff, features); `spectrum` (optional, float64 [total_length]) receives d."""
    L = _llib()
    dev = signal.device
    if coeff is None:
        coeff = torch.empty(batch.total_length, dtype=torch.float64, device=dev)
    if features is None:
        features = torch.empty((batch.count, 72), dtype=torch.float32, device=dev)
    _check(L.ht_batch_features(batch.handle, _p(signal, "signal", torch.float64), _p(psf, "psf", torch.float64),
                               _p(coeff, "coeff", torch.float64), _p(features, "features", torch.float32),
                               _p(spectrum, "spectrum", torch.float64), _stream()), "ht_batch_features")
    return coeff, features


def ht_batch_restore_learned(batch, coeff, psf, norm, mu_grid, pred, cert_half=8, G=None, kb=None, mb=None,
                             fallback=None, spectrum=None):
    """coeff (from ht_batch_features) is overwritten with the restorations; `spectrum`
    is the feature pass's eigenvalue output (or None: recomputed)."""
    L = _llib()
    dev = coeff.device
    K = mu_grid.shape[-1]
    kb = torch.empty(batch.count, dtype=torch.int32, device=dev) if kb is None else kb
    mb = torch.empty(batch.count, dtype=torch.float64, device=dev) if mb is None else mb
    fallback = torch.empty(batch.count, dtype=torch.int32, device=dev) if fallback is None else fallback
    _check(L.ht_batch_restore_learned(batch.handle, _p(coeff, "coeff", torch.float64), _p(psf, "psf", torch.float64),
                                      _p(spectrum, "spectrum", torch.float64), NORMS.get(norm, norm), _p(mu_grid, "mu_grid", torch.float64), int(K),
                                      _p(pred, "pred", torch.float32), int(cert_half), _p(G, "G", torch.float64),
                                      _p(kb, "k_best", torch.int32), _p(mb, "mu_best", torch.float64),
                                      _p(fallback, "fallback", torch.int32), _stream()), "ht_batch_restore_learned")
    return coeff, kb, mb, fallback


def ht_gemm_bf16(M, N, K, A, sa, B, sb, bias=None, act=0, Z=None, C=None, Cb=None, ldc=None):
    """C = act(A B + bias); A(i,k) = A[i sa[0] + k sa[1]], B(k,j) = B[k sb[0] + j sb[1]]."""
    L = _llib()
    _check(L.ht_gemm_bf16(int(M), int(N), int(K), _p(A, "A", BF16), int(sa[0]), int(sa[1]), _p(B, "B", BF16),
                          int(sb[0]), int(sb[1]), _p(bias, "bias", torch.float32), int(act),
                          _p(Z, "Z", torch.float32), _p(C, "C", torch.float32), int(ldc if ldc is not None else N),
                          _p(Cb, "Cb", BF16), _stream()), "ht_gemm_bf16")


def ht_to_bf16(src, dst, rows, cols, mean=None, std=None):
    _check(_llib().ht_to_bf16(_p(src, "src", torch.float32), _p(dst, "dst", BF16), int(rows), int(cols),
                              _p(mean, "mean", torch.float32), _p(std, "std", torch.float32), _stream()),
           "ht_to_bf16")


def ht_from_bf16(src, dst):
    _check(_llib().ht_from_bf16(_p(src, "src", BF16), _p(dst, "dst", torch.float32), src.numel(), _stream()),
           "ht_from_bf16")


def ht_gelu_backward(z, dh, dz, dzb=None):
    _check(_llib().ht_gelu_backward(_p(z, "z", torch.float32), _p(dh, "dh", torch.float32),
                                    _p(dz, "dz", torch.float32), _p(dzb, "dzb", BF16), z.numel(), _stream()),
           "ht_gelu_backward")


def ht_colsum(X, rows, cols, out, weight=None):
    _check(_llib().ht_colsum(_p(X, "X", torch.float32), int(rows), int(cols), _p(weight, "weight", torch.float32),
                             _p(out, "out", torch.float32), _stream()), "ht_colsum")


def ht_mse_grad(y, t, dy, sq):
    _check(_llib().ht_mse_grad(_p(y, "y", torch.float32), _p(t, "t", torch.float32), _p(dy, "dy", torch.float32),
                               _p(sq, "sq", torch.float32), y.numel(), _stream()), "ht_mse_grad")


def ht_outer(dy, w, dh, rows, cols):
    _check(_llib().ht_outer(_p(dy, "dy", torch.float32), _p(w, "w", torch.float32), _p(dh, "dh", torch.float32),
                            int(rows), int(cols), _stream()), "ht_outer")


def ht_adam(p, g, m, v, lr, step, pb=None, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(_llib().ht_adam(_p(p, "p", torch.float32), _p(g, "g", torch.float32), _p(m, "m", torch.float32),
                           _p(v, "v", torch.float32), p.numel(), float(lr), float(beta1), float(beta2), float(eps),
                           int(step), _p(pb, "pb", BF16), _stream()), "ht_adam")


# ----------------------------------------------------------------------------- the network object

MLP_PARAMS_VEC, MLP_GRADS_VEC, MLP_ADAM_M_VEC, MLP_ADAM_V_VEC, MLP_MEAN_VEC, MLP_STD_VEC = range(6)


class Mlp:
    """The learned-mu network owned by the library (ht_mlp_create): parameters, Adam state,
    standardisation and activation buffers for up to `max_rows` rows."""

    def __init__(self, max_rows):
        L = _llib()
        h = ctypes.c_void_p()
        _check(L.ht_mlp_create(int(max_rows), ctypes.byref(h)), "ht_mlp_create")
        self._h = h
        self.max_rows = int(max_rows)
        self.param_count = int(L.ht_mlp_param_count())

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            _check(_llib().ht_mlp_destroy(self._h), "ht_mlp_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def steps(self):
        return int(_llib().ht_mlp_steps(self._h))

    def get(self, which, out=None):
        n = 72 if which in (MLP_MEAN_VEC, MLP_STD_VEC) else self.param_count
        out = torch.empty(n, dtype=torch.float32, device="cuda") if out is None else out
        _check(_llib().ht_mlp_get(self._h, int(which), _p(out, "out", torch.float32), _stream()), "ht_mlp_get")
        return out


def ht_mlp_set_params(mlp, params):
    _check(_llib().ht_mlp_set_params(mlp.handle, _p(params, "params", torch.float32), _stream()), "ht_mlp_set_params")


def ht_mlp_set_state(mlp, adam_m=None, adam_v=None, steps=0, mean=None, std=None):
    _check(_llib().ht_mlp_set_state(mlp.handle, _p(adam_m, "adam_m", torch.float32), _p(adam_v, "adam_v", torch.float32),
                                    int(steps), _p(mean, "mean", torch.float32), _p(std, "std", torch.float32),
                                    _stream()), "ht_mlp_set_state")


def ht_mlp_fit_standardisation(mlp, features):
    _check(_llib().ht_mlp_fit_standardisation(mlp.handle, _p(features, "features", torch.float32),
                                              int(features.shape[0]), _stream()), "ht_mlp_fit_standardisation")


def ht_mlp_forward(mlp, features, pred=None):
    rows = int(features.shape[0])
    _check(_llib().ht_mlp_forward(mlp.handle, _p(features, "features", torch.float32), rows,
                                  _p(pred, "pred", torch.float32), _stream()), "ht_mlp_forward")
    return pred


def ht_mlp_predict(mlp, features, pred=None):
    rows = int(features.shape[0])
    pred = torch.empty(rows, dtype=torch.float32, device=features.device) if pred is None else pred
    _check(_llib().ht_mlp_predict(mlp.handle, _p(features, "features", torch.float32), rows,
                                  _p(pred, "pred", torch.float32), _stream()), "ht_mlp_predict")
    return pred


def ht_mlp_backward(mlp, target, loss=None):
    _check(_llib().ht_mlp_backward(mlp.handle, _p(target, "target", torch.float32), int(target.shape[0]),
                                   _p(loss, "loss", torch.float32), _stream()), "ht_mlp_backward")


def ht_mlp_adam_step(mlp, lr):
    _check(_llib().ht_mlp_adam_step(mlp.handle, float(lr), _stream()), "ht_mlp_adam_step")


def ht_mlp_train_step(mlp, features, target, idx, lr, loss=None):
    _check(_llib().ht_mlp_train_step(mlp.handle, _p(features, "features", torch.float32),
                                     _p(target, "target", torch.float32), _p(idx, "idx", torch.int32),
                                     int(idx.shape[0]), float(lr), _p(loss, "loss", torch.float32), _stream()),
           "ht_mlp_train_step")


def ht_mlp_weights_of(mlp):
    w = MlpWeights()
    _check(_llib().ht_mlp_weights_of(mlp.handle, ctypes.byref(w)), "ht_mlp_weights_of")
    return w


def ht_log10_labels(mu, labels=None):
    labels = torch.empty(mu.shape, dtype=torch.float32, device=mu.device) if labels is None else labels
    _check(_llib().ht_log10_labels(_p(mu, "mu", torch.float64), _p(labels, "labels", torch.float32), mu.numel(),
                                   _stream()), "ht_log10_labels")
    return labels


def ht_lambda_predict(batch, mlp, signal, psf, coeff=None, features=None, spectrum=None, pred=None):
    """Returns (pred, coeff, features): predicted log10 mu per signal, with the feature
    pass's coefficients and features."""
    L = _llib()
    dev = signal.device
    coeff = torch.empty(batch.total_length, dtype=torch.float64, device=dev) if coeff is None else coeff
    features = torch.empty((batch.count, 72), dtype=torch.float32, device=dev) if features is None else features
    pred = torch.empty(batch.count, dtype=torch.float32, device=dev) if pred is None else pred
    _check(L.ht_lambda_predict(batch.handle, mlp.handle, _p(signal, "signal", torch.float64),
                               _p(psf, "psf", torch.float64), _p(coeff, "coeff", torch.float64),
                               _p(features, "features", torch.float32), _p(spectrum, "spectrum", torch.float64),
                               _p(pred, "pred", torch.float32), _stream()), "ht_lambda_predict")
    return pred, coeff, features
