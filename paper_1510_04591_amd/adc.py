"""ctypes binding of libadc.so (the C ABI in include/adc.h).

Argument marshalling only: every function forwards to the C entry point of
the same name.  Device arrays are passed as torch tensors (their data_ptr())
or raw integer addresses.  The library is loaded on first use; a missing
library raises ImportError (there is no fallback path).
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ADC_LIB", os.path.join(_HERE, "libadc.so"))

ADC_OK = 0
ADC_ERR_ARG = 1
ADC_ERR_NOMEM = 2
ADC_ERR_HIP = 3
ADC_ERR_NOCONV = 4
ADC_ERR_ACCURACY = 5
ADC_ERR_UNSUPPORTED = 6

ADC_RANK_BOUND = 0
ADC_RANK_MLP = 1
ADC_RANK_FIXED = 2
ADC_SAMPLE_DIRECT = 0
ADC_SAMPLE_FMM = 1

MLP_NPARAM = 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1


class adc_opts(C.Structure):
    _fields_ = [
        ("dc_leaf", C.c_int32), ("hss_min_k", C.c_int32), ("hss_levels", C.c_int32),
        ("hss_leaf", C.c_int32), ("id_tol", C.c_double), ("oversample", C.c_int32),
        ("rank_mode", C.c_int32), ("fixed_rank", C.c_int32), ("max_retries", C.c_int32),
        ("max_iter", C.c_int32), ("seed", C.c_uint64), ("force_dense", C.c_int32),
        ("strict", C.c_int32), ("check_tol", C.c_double), ("nprobe", C.c_int32),
        ("shift_max", C.c_int32), ("shift_thresh", C.c_double), ("r_cap", C.c_int32),
        ("rank_eps", C.c_double), ("hss_min_flops", C.c_double), ("sample_mode", C.c_int32),
        ("fmm_order", C.c_int32), ("sat_guard", C.c_int32),
        ("batch_bytes", C.c_double),
    ]


class adc_report(C.Structure):
    _fields_ = [
        ("levels", C.c_int32), ("merges", C.c_int32), ("hss_merges", C.c_int32),
        ("retries", C.c_int32), ("hss_fallbacks", C.c_int32), ("info_index", C.c_int32),
        ("n_per_level", C.c_int64 * 64), ("K_per_level", C.c_int64 * 64),
        ("hss_per_level", C.c_int32 * 64), ("max_rank", C.c_int32), ("samples", C.c_int32),
        ("t_phase", C.c_double * 12), ("phase_flops", C.c_double * 12), ("phase_bytes", C.c_double * 12),
        ("phase_launches", C.c_int32 * 12), ("flops_model", C.c_double), ("bytes_model", C.c_double),
        ("check_err_max", C.c_double),
        ("kern_time", C.c_double * 12), ("kern_flops", C.c_double * 12), ("kern_bytes", C.c_double * 12),
        ("kern_launches", C.c_int32 * 12), ("hss_saturated", C.c_int32), ("hss_sat_nodes", C.c_int32),
    ]

    KERNELS = ("k_gemm_f64", "k_gemm_f64_n64", "k_hss_sample", "k_pack_rot", "k_secular", "k_hss_compress",
               "k_gemm_f64_big", "k_gemm_f64_n96", "k_fmm_leaf", "k_fmm_m2l", "unused10", "unused11")

    def as_dict(self):
        L = self.levels
        return dict(levels=L, merges=self.merges, hss_merges=self.hss_merges, retries=self.retries,
                    hss_fallbacks=self.hss_fallbacks, info_index=self.info_index,
                    n_per_level=list(self.n_per_level[:L]), K_per_level=list(self.K_per_level[:L]),
                    hss_per_level=list(self.hss_per_level[:L]), max_rank=self.max_rank,
                    samples=self.samples, t_phase=list(self.t_phase), phase_flops=list(self.phase_flops),
                    phase_bytes=list(self.phase_bytes), phase_launches=list(self.phase_launches),
                    flops_model=self.flops_model,
                    bytes_model=self.bytes_model, check_err_max=self.check_err_max,
                    kern_time=list(self.kern_time), kern_flops=list(self.kern_flops),
                    kern_bytes=list(self.kern_bytes), kern_launches=list(self.kern_launches),
                    hss_saturated=self.hss_saturated, hss_sat_nodes=self.hss_sat_nodes)


class AdcError(RuntimeError):
    def __init__(self, status, where, report=None):
        self.status = status
        self.report = report
        super().__init__(f"{where}: {status_string(status)}")


_lib = None
_P = C.c_void_p
_I64 = C.c_int64
_I32 = C.c_int32
_D = C.c_double

_SIGS = {
    "adc_create": (C.POINTER(_P), C.c_int, _P),
    "adc_destroy": (_P,),
    "adc_opts_default": (C.POINTER(adc_opts),),
    "adc_workspace_query": (_P, _I64, C.POINTER(adc_opts), C.POINTER(C.c_size_t)),
    "adc_stedc": (_P, _I64, _P, _P, _P, _P, _I64, _P, C.c_size_t, C.POINTER(adc_opts), C.POINTER(adc_report)),
    "adc_stedc_batched": (_P, _I32, C.POINTER(_I64), C.POINTER(_P), C.POINTER(_P), C.POINTER(_P),
                          C.POINTER(_P), C.POINTER(_I64), C.POINTER(adc_opts), C.POINTER(adc_report)),
    "adc_secular": (_P, _I64, _P, _P, _D, _P, _P, _P),
    "adc_lowner": (_P, _I64, _P, _P, _D, _P, _P, _P, _P),
    "adc_cauchy_gemm": (_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _I64, _P, _I64),
    "adc_cauchy_gemm_noalloc": (_P, _I64, _I64, _P, _P, _P, _P, _P, _P, _I64, _P, _I64),
    "adc_hss_build": (_P, _I64, _P, _P, _P, _P, _P, _P, _I32, C.POINTER(adc_opts), C.POINTER(_P)),
    "adc_hss_apply": (_P, _P, _I64, _P, _I64, _P, _I64),
    "adc_rank_estimate": (_P, _I64, _P, _P, _P, C.POINTER(adc_opts), C.POINTER(_I32), C.POINTER(_I32), _I32,
                          C.POINTER(_I32)),
    "adc_hss_sample": (_P, _I64, _P, _P, _P, _P, _P, _P, _I32, C.POINTER(adc_opts), _P, _P),
    "adc_hss_info": (_P, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32),
                     C.POINTER(_I32), C.POINTER(_D)),
    "adc_hss_free": (_P,),
    "adc_hss_nodes": (_P, _I32, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32),
                      C.POINTER(_I32)),
    "adc_mlp_features": (_P, _I64, _P, _P, _P, C.POINTER(_I64), _I32, _P),
    "adc_mlp_init": (_P, C.c_uint64),
    "adc_mlp_train": (_P, _I32, _P, _P, _I32, _I32, C.c_float, C.POINTER(C.c_float)),
    "adc_mlp_infer": (_P, _I32, _P, _P),
    "adc_mlp_grad": (_P, _I32, _P, _P, _P, C.POINTER(C.c_float)),
    "adc_mlp_get": (_P, _P),
    "adc_mlp_set": (_P, _P),
    "adc_mlp_collect": (_P, _I64, _P, _P, _P, _P, _I64, C.POINTER(adc_opts), _I64, _P, _P, C.POINTER(_I64)),
}
EXPORTS = tuple(_SIGS) + ("adc_status_string",)


def lib():
    """The loaded library (raises ImportError when it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libadc.so not found at {LIB_PATH}: build it with python -m paper_1510_04591_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = list(args)
            f.restype = C.c_int
        L.adc_status_string.argtypes = [C.c_int]
        L.adc_status_string.restype = C.c_char_p
        _lib = L
    return _lib


def status_string(s):
    return lib().adc_status_string(int(s)).decode()


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _check(s, where, report=None):
    if s != ADC_OK:
        raise AdcError(s, where, report)


def opts(**kw):
    """adc_opts with the library defaults, updated by keyword."""
    o = adc_opts()
    _check(lib().adc_opts_default(C.byref(o)), "adc_opts_default")
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


# ------------------------------------------------------------ raw entry points
def adc_create(device=0, stream=None):
    h = _P()
    _check(lib().adc_create(C.byref(h), int(device), stream), "adc_create")
    return h


def adc_destroy(ctx):
    _check(lib().adc_destroy(ctx), "adc_destroy")


def adc_workspace_query(ctx, n, o=None):
    b = C.c_size_t()
    _check(lib().adc_workspace_query(ctx, int(n), C.byref(o) if o is not None else None, C.byref(b)),
           "adc_workspace_query")
    return b.value


def adc_stedc(ctx, n, diag, offdiag, w, Z, ldz, ws=None, ws_bytes=0, o=None, rep=None):
    return lib().adc_stedc(ctx, int(n), _ptr(diag), _ptr(offdiag), _ptr(w), _ptr(Z), int(ldz), _ptr(ws),
                           int(ws_bytes), C.byref(o) if o is not None else None,
                           C.byref(rep) if rep is not None else None)


def adc_stedc_batched(ctx, ns, diags, offs, ws, Zs, ldzs, o=None, rep=None):
    cnt = len(ns)
    arr = lambda xs: (_P * cnt)(*[_ptr(x) for x in xs])
    return lib().adc_stedc_batched(ctx, cnt, (_I64 * cnt)(*ns), arr(diags), arr(offs), arr(ws), arr(Zs),
                                   (_I64 * cnt)(*ldzs), C.byref(o) if o is not None else None,
                                   C.byref(rep) if rep is not None else None)


def adc_secular(ctx, K, d, z, rho, lam, gam, mu):
    return lib().adc_secular(ctx, int(K), _ptr(d), _ptr(z), float(rho), _ptr(lam), _ptr(gam), _ptr(mu))


def adc_lowner(ctx, K, d, z, rho, gam, mu, uh, v):
    return lib().adc_lowner(ctx, int(K), _ptr(d), _ptr(z), float(rho), _ptr(gam), _ptr(mu), _ptr(uh), _ptr(v))


def adc_cauchy_gemm(ctx, P, K, d, gam, mu, uh, v, X, ldx, Y, ldy):
    return lib().adc_cauchy_gemm(ctx, int(P), int(K), _ptr(d), _ptr(gam), _ptr(mu), _ptr(uh), _ptr(v),
                                 _ptr(X), int(ldx), _ptr(Y), int(ldy))


def adc_cauchy_gemm_noalloc(ctx, P, K, d, gam, mu, uh, v, X, ldx, Y, ldy):
    return lib().adc_cauchy_gemm_noalloc(ctx, int(P), int(K), _ptr(d), _ptr(gam), _ptr(mu), _ptr(uh), _ptr(v),
                                         _ptr(X), int(ldx), _ptr(Y), int(ldy))


def adc_hss_build(ctx, K, d, gam, mu, uh, v, omega, s, o=None):
    h = _P()
    st = lib().adc_hss_build(ctx, int(K), _ptr(d), _ptr(gam), _ptr(mu), _ptr(uh), _ptr(v), _ptr(omega), int(s),
                             C.byref(o) if o is not None else None, C.byref(h))
    return st, h


def adc_hss_sample(ctx, K, d, gam, mu, uh, v, omega, s, o, phi, theta):
    return lib().adc_hss_sample(ctx, int(K), _ptr(d), _ptr(gam), _ptr(mu), _ptr(uh), _ptr(v), _ptr(omega), int(s),
                                C.byref(o) if o is not None else None, _ptr(phi), _ptr(theta))


def adc_rank_estimate(ctx, K, d, gam, mu, o=None, cap=1 << 16):
    """(status, r, moved leaf boundaries) of the library's rank estimate."""
    r = _I32()
    nb = _I32()
    arr = (_I32 * cap)()
    st = lib().adc_rank_estimate(ctx, int(K), _ptr(d), _ptr(gam), _ptr(mu), C.byref(o) if o is not None else None,
                                 C.byref(r), arr, int(cap), C.byref(nb))
    return st, r.value, [arr[i] for i in range(min(nb.value, cap))] if st == 0 else []


def adc_hss_apply(ctx, h, P, X, ldx, Y, ldy):
    return lib().adc_hss_apply(ctx, h, int(P), _ptr(X), int(ldx), _ptr(Y), int(ldy))


def adc_hss_info(h):
    vals = [_I32(), _I32(), _I32(), _I32(), _I32(), _D()]
    st = lib().adc_hss_info(h, *[C.byref(v) for v in vals])
    _check(st, "adc_hss_info")
    return dict(levels=vals[0].value, leaves=vals[1].value, max_rank=vals[2].value, samples=vals[3].value,
                retries=vals[4].value, check_err=vals[5].value)


def adc_hss_free(h):
    return lib().adc_hss_free(h)


def adc_hss_nodes(h, nmax=1 << 16):
    arrs = [(_I32 * nmax)() for _ in range(4)]
    cnt = _I32()
    _check(lib().adc_hss_nodes(h, nmax, *arrs, C.byref(cnt)), "adc_hss_nodes")
    n = min(cnt.value, nmax)
    return [dict(lo=arrs[0][i], hi=arrs[1][i], kr=arrs[2][i], kc=arrs[3][i]) for i in range(n)]


def adc_mlp_features(ctx, K, d, gam, mu, bounds, feat):
    nb = len(bounds) - 2
    return lib().adc_mlp_features(ctx, int(K), _ptr(d), _ptr(gam), _ptr(mu), (_I64 * len(bounds))(*bounds),
                                  int(nb), _ptr(feat))


def adc_mlp_init(ctx, seed):
    return lib().adc_mlp_init(ctx, int(seed))


def adc_mlp_train(ctx, B, X, y, epochs, batch, lr):
    loss = C.c_float()
    st = lib().adc_mlp_train(ctx, int(B), _ptr(X), _ptr(y), int(epochs), int(batch), float(lr), C.byref(loss))
    return st, loss.value


def adc_mlp_infer(ctx, B, X, y):
    return lib().adc_mlp_infer(ctx, int(B), _ptr(X), _ptr(y))


def adc_mlp_grad(ctx, B, X, y, g):
    loss = C.c_float()
    st = lib().adc_mlp_grad(ctx, int(B), _ptr(X), _ptr(y), _ptr(g), C.byref(loss))
    return st, loss.value


def adc_mlp_get(ctx, params):
    return lib().adc_mlp_get(ctx, _ptr(params))


def adc_mlp_set(ctx, params):
    return lib().adc_mlp_set(ctx, _ptr(params))


def adc_mlp_collect(ctx, n, diag, offdiag, w, Z, ldz, o, max_rows, X, y):
    rows = _I64()
    st = lib().adc_mlp_collect(ctx, int(n), _ptr(diag), _ptr(offdiag), _ptr(w), _ptr(Z), int(ldz),
                               C.byref(o) if o is not None else None, int(max_rows), _ptr(X), _ptr(y),
                               C.byref(rows))
    return st, rows.value


# ------------------------------------------------------------ convenience
class Context:
    """A library context on the current torch device and stream."""

    def __init__(self, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        dev = torch.cuda.current_device() if device is None else int(device)
        s = torch.cuda.current_stream(dev) if stream is None else stream
        self.device = dev
        self.stream = s
        self.h = adc_create(dev, s.cuda_stream)

    def close(self):
        if self.h:
            adc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eigh_tridiagonal(ctx, diag, offdiag, **kw):
    """(w, Z, report) of the tridiagonal matrix (diag, offdiag) on the GPU.

    diag, offdiag: float64 CUDA tensors.  Z is returned column-major as the
    transpose of a row-major buffer (Z[:, j] is the eigenvector of w[j])."""
    import torch
    n = diag.shape[0]
    dev = diag.device
    w = torch.empty(n, dtype=torch.float64, device=dev)
    Zt = torch.empty((n, n), dtype=torch.float64, device=dev)
    o = opts(**kw)
    rep = adc_report()
    s = adc_stedc(ctx.h, n, diag, offdiag if n > 1 else None, w, Zt, n, None, 0, o, rep)
    _check(s, "adc_stedc", rep.as_dict())
    return w, Zt.t(), rep.as_dict()
