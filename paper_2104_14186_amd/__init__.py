"""Python binding of libqdwhp.so (QDWHpartial-EIG / -SVD on MI355X).

Argument marshalling only: torch supplies device memory and the current
stream; every step of the solve runs in the HIP library.  Importing this
package does not need a GPU; calling it does, and fails loudly when the
library has not been built.
"""
import ctypes
import math
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqdwhp.so")
_lib = None

LARGEST, SMALLEST = 0, 1
FP64, MIXED_FP32 = 0, 1
KIND_AUTO, KIND_QR, KIND_CHOL = 0, 1, 2
STATUS = {0: "OK", 1: "NONFINITE", 2: "NO_SUBSPACE", 3: "CHOL", 4: "WORKSPACE",
          5: "HIP", 6: "NOCONV"}


class QdwhpError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: status {status} ({STATUS.get(status, 'invalid argument')})")


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("s_eig", ctypes.c_double),
                ("eig_iters", ctypes.c_int), ("kappa_max", ctypes.c_double),
                ("svd_qr_first", ctypes.c_int), ("precision", ctypes.c_int),
                ("polish_steps", ctypes.c_int), ("seed", ctypes.c_uint64),
                ("lanczos_vectors", ctypes.c_int), ("lanczos_steps", ctypes.c_int),
                ("tau", ctypes.c_double), ("mu", ctypes.c_double), ("rho", ctypes.c_double),
                ("alpha", ctypes.c_double), ("s_svd", ctypes.c_double),
                ("kinds", ctypes.c_int * 16), ("graphs", ctypes.c_int),
                ("tau_policy", ctypes.c_int), ("use_omega", ctypes.c_int), ("zolo_r", ctypes.c_int)]


Opts._field_names = frozenset(f for f, _ in Opts._fields_)


class Info(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int64), ("ell", ctypes.c_int64), ("ind", ctypes.c_int64),
                ("n_above", ctypes.c_int64),
                ("tau", ctypes.c_double), ("mu", ctypes.c_double), ("rho", ctypes.c_double),
                ("alpha", ctypes.c_double), ("s", ctypes.c_double),
                ("lmax", ctypes.c_double), ("lmin", ctypes.c_double),
                ("n_iter", ctypes.c_int), ("kinds", ctypes.c_int * 16),
                ("weights", (ctypes.c_double * 3) * 16), ("retries", ctypes.c_int),
                ("jacobi_sweeps", ctypes.c_int), ("ms", ctypes.c_double * 8),
                ("flops_table1", ctypes.c_double), ("status", ctypes.c_int),
                ("rr_split", ctypes.c_int64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_
             if f not in ("kinds", "weights", "ms")}
        d["kinds"] = ["qr" if x == KIND_QR else "chol" for x in list(self.kinds)[:self.n_iter]]
        d["weights"] = [tuple(self.weights[i]) for i in range(self.n_iter)]
        d["ms"] = list(self.ms)
        return d


class Problem(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int), ("which", ctypes.c_int),
                ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64),
                ("fraction", ctypes.c_double), ("k", ctypes.c_int64),
                ("w", ctypes.c_void_p), ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64),
                ("V", ctypes.c_void_p), ("ldv", ctypes.c_int64)]


PROBLEM_EIG, PROBLEM_SVD = 0, 1
PENDING = 100
TUNING_PATH = os.path.join(_PKG, "tuning_gfx950.json")

_P, _I64, _D, _I, _SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_size_t
_PP = ctypes.POINTER(ctypes.c_void_p)
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PD = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "qdwhp_opts_default": (None, [ctypes.POINTER(Opts)]),
    "qdwhp_strerror": (ctypes.c_char_p, [_I]),
    "qdwhp_zolo_coeffs": (_I, [_D, _I, _PD, _PD, _PD, _PD]),
    "qdwhp_heig_workspace": (_SZ, [_I64, _D, ctypes.POINTER(Opts)]),
    "qdwhp_heig": (_I, [_P, _I64, _I64, _D, _I, _P, _P, _I64, _P, _SZ,
                        ctypes.POINTER(Opts), _P, ctypes.POINTER(Info)]),
    "qdwhp_eig_workspace": (_SZ, [_I64, _D, ctypes.POINTER(Opts)]),
    "qdwhp_eig_count": (_I64, [_I64, _D]),
    "qdwhp_svd_workspace": (_SZ, [_I64, _I64, _I64, ctypes.POINTER(Opts)]),
    "qdwhp_eig": (_I, [_P, _I64, _I64, _D, _I, _P, _P, _I64, _P, _SZ,
                       ctypes.POINTER(Opts), _P, ctypes.POINTER(Info)]),
    "qdwhp_svd": (_I, [_P, _I64, _I64, _I64, _I64, _P, _I64, _P, _P, _I64, _P, _SZ,
                       ctypes.POINTER(Opts), _P, ctypes.POINTER(Info)]),
    "qdwhp_dgemm": (_I, [_I, _I, _I64, _I64, _I64, _D, _P, _I64, _P, _I64, _D, _P, _I64, _I, _P]),
    "qdwhp_spd_inverse_workspace": (_SZ, [_I64]),
    "qdwhp_spd_inverse": (_I, [_P, _I64, _I64, _P, _SZ, _P]),
    "qdwhp_geqrf_workspace": (_SZ, [_I64, _I64]),
    "qdwhp_geqrf": (_I, [_P, _I64, _I64, _I64, _P, _P, _SZ, _P]),
    "qdwhp_orgqr": (_I, [_P, _I64, _I64, _I64, _P, _I64, _I64, _P, _I64, _P, _SZ, _P]),
    "qdwhp_syev_workspace": (_SZ, [_I64]),
    "qdwhp_syev": (_I, [_P, _I64, _I64, _P, _P, _I64, _P, _SZ, _P, ctypes.POINTER(_I)]),
    "qdwhp_syev_dc_workspace": (_SZ, [_I64]),
    "qdwhp_syev_dc": (_I, [_P, _I64, _I64, _P, _P, _I64, _P, _SZ, _P, ctypes.POINTER(_I)]),
    "qdwhp_gesvj_workspace": (_SZ, [_I64]),
    "qdwhp_gesvj": (_I, [_P, _I64, _I64, _P, _P, _I64, _P, _SZ, _P, ctypes.POINTER(_I)]),
    "qdwhp_problem_workspace": (_SZ, [ctypes.POINTER(Problem), ctypes.POINTER(Opts)]),
    "qdwhp_batched_workspace": (_SZ, [_I, ctypes.POINTER(Problem), ctypes.POINTER(Opts)]),
    "qdwhp_batched": (_I, [_I, ctypes.POINTER(Problem), _P, _SZ, ctypes.POINTER(Opts), _I, _P,
                           ctypes.POINTER(Info), ctypes.POINTER(_I)]),
    "qdwhp_dgemm_grouped_workspace": (_SZ, [_I]),
    "qdwhp_dgemm_grouped": (_I, [_I, _I, _I, _PI64, _PI64, _PI64, _PD, _PP, _PI64, _PP, _PI64, _PD,
                                 _PP, _PI64, _P, _SZ, _P]),
    "qdwhp_serve_create": (_I, [_SZ, _I, ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_void_p)]),
    "qdwhp_serve_submit": (_I, [_P, ctypes.POINTER(Problem), _PI64]),
    "qdwhp_serve_poll": (_I, [_P, _I64, _I, ctypes.POINTER(Info), _PD, _PD]),
    "qdwhp_serve_destroy": (_I, [_P]),
    "qdwhp_serve_stats": (_I, [_P, ctypes.POINTER(_SZ), ctypes.POINTER(_SZ), ctypes.POINTER(_I), _PI64, _PI64, _I]),
    "qdwhp_noalloc_max_bytes": (_SZ, []),
    "qdwhp_eig_noalloc": (_I, [_P, _I64, _I64, _D, _I, _P, _P, _I64, ctypes.POINTER(Opts), _P,
                               ctypes.POINTER(Info)]),
    "qdwhp_tune_set": (_I, [ctypes.c_char_p, _I64]),
    "qdwhp_tune_get": (_I64, [ctypes.c_char_p, _I64]),
    "qdwhp_tune_get_sized": (_I64, [ctypes.c_char_p, _I64, _I64]),
    "qdwhp_tune_clear": (None, []),
    "qdwhp_graphs_clear": (_I, []),
    "qdwhp_graphs_count": (_I64, []),
    "qdwhp_profile_begin": (None, []),
    "qdwhp_profile_end": (_I, [ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_I64)]),
}


def lib():
    """Load libqdwhp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                               "(hipcc for gfx950) first; there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        load_tuning()
    return _lib


def load_tuning(path=TUNING_PATH):
    """Apply the autotuner's table (JSON {"params": {key: int}}) if present."""
    import json
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        params = json.load(f).get("params", {})
    for key, v in params.items():
        tune_set(key, int(v))
    return params


def tune_set(key, value):
    _check(lib().qdwhp_tune_set(key.encode(), int(value)), "qdwhp_tune_set")


def tune_get(key, fallback=-1):
    return lib().qdwhp_tune_get(key.encode(), int(fallback))


def exported_symbols():
    return list(_SIGS)


def default_opts(**kw):
    o = Opts()
    lib().qdwhp_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "kinds":
            for i, x in enumerate(v):
                o.kinds[i] = {"qr": KIND_QR, "chol": KIND_CHOL, "auto": KIND_AUTO}.get(x, x)
        elif k in Opts._field_names:
            setattr(o, k, v)
        else:
            raise KeyError(f"qdwhp_opts has no field {k!r}")
    return o


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check(st, where):
    if st != 0:
        raise QdwhpError(st, where)


def _colmajor(A):
    """Column-major copy of a 2-D float64 CUDA tensor: returns (buffer, ld)
    where buffer is a contiguous (cols, rows) tensor holding A column by column."""
    return A.t().contiguous(), A.shape[0]


def _workspace(torch, nbytes, device):
    return torch.empty(max(1, (nbytes + 7) // 8), dtype=torch.float64, device=device)


def dgemm(A, B, C=None, alpha=1.0, beta=0.0, transa=False, transb=False, upper=False, f32=False):
    """C = alpha op(A) op(B) + beta C on column-major views.

    A, B, C are 2-D float64 CUDA tensors given as column-major buffers, i.e.
    contiguous tensors of shape (cols, rows) (the transpose of the logical
    matrix).  Returns C in the same convention.
    """
    import torch
    ka, ma = A.shape          # logical A is ma x ka (column-major buffer of shape (ka, ma))
    kb, mb = B.shape
    m, k = (ka, ma) if transa else (ma, ka)
    kk, n = (kb, mb) if transb else (mb, kb)
    assert k == kk
    if C is None:
        C = torch.zeros((n, m), dtype=torch.float64, device=A.device)
    st = lib().qdwhp_dgemm(int(transa), int(transb), m, n, k, alpha, _ptr(A), ma, _ptr(B), mb,
                           beta, _ptr(C), m, int(upper) | (2 if f32 else 0), _stream(torch))
    _check(st, "qdwhp_dgemm")
    return C


def _info_dict(info):
    return info.as_dict()


def _count(n, fraction, where="qdwhp_eig"):
    """k for this n and fraction, as the library computes it; the library's
    own status for the argument it would reject (n: -2, fraction: -4)."""
    kk = int(lib().qdwhp_eig_count(n, float(fraction)))
    if kk < 1:
        raise QdwhpError(-2 if n < 1 else -4, where)
    return kk


def _sym_storage(A):
    """Column-major storage of the symmetric A.  A dense tensor in either
    order holds the same matrix (row-major storage of A is column-major
    storage of A^T = A), so it is passed as it is; other strides are
    copied."""
    if A.is_contiguous() or A.t().is_contiguous():
        return A
    return A.t().contiguous()


def eig(A, fraction=None, k=None, which="largest", opts=None, return_info=False, stream=None):
    """Wanted eigenpairs of the symmetric n x n float64 CUDA tensor A (QDWHpartial-EIG).

    A dense A (either memory order) is read in place, without a copy; A must
    be symmetric, as the method assumes (its two triangles are both read).

    Returns (w, V) with w (k,) most wanted first and V (n, k); with
    return_info=True also the solver report as a dict.
    """
    import torch
    n = A.shape[0]
    assert A.shape == (n, n) and A.dtype == torch.float64 and A.is_cuda
    if fraction is None:
        fraction = float(k) / n
    kk = _count(n, fraction)
    o = opts if opts is not None else default_opts()
    Acm = _sym_storage(A)
    nbytes = lib().qdwhp_eig_workspace(n, fraction, ctypes.byref(o))
    ws = _workspace(torch, nbytes, A.device)
    w = torch.empty(kk, dtype=torch.float64, device=A.device)
    Vb = torch.empty((kk, n), dtype=torch.float64, device=A.device)
    info = Info()
    st = lib().qdwhp_eig(_ptr(Acm), n, n, fraction, SMALLEST if which == "smallest" else LARGEST,
                         _ptr(w), _ptr(Vb), n, _ptr(ws), nbytes, ctypes.byref(o),
                         stream if stream is not None else _stream(torch), ctypes.byref(info))
    _check(st, "qdwhp_eig")
    out = (w, Vb.t())
    return out + (info.as_dict(),) if return_info else out


def eig_noalloc(A, fraction=None, k=None, which="largest", opts=None, return_info=False, stream=None):
    """qdwhp_eig_noalloc: eig() with the library's fixed workspace array (no
    workspace is allocated; n limited by qdwhp_noalloc_max_bytes).  The
    outputs are allocated here, as for eig()."""
    import torch
    n = A.shape[0]
    assert A.shape == (n, n) and A.dtype == torch.float64 and A.is_cuda
    if fraction is None:
        fraction = float(k) / n
    kk = _count(n, fraction)
    o = opts if opts is not None else default_opts()
    Acm = _sym_storage(A)
    w = torch.empty(kk, dtype=torch.float64, device=A.device)
    Vb = torch.empty((kk, n), dtype=torch.float64, device=A.device)
    info = Info()
    st = lib().qdwhp_eig_noalloc(_ptr(Acm), n, n, fraction, SMALLEST if which == "smallest" else LARGEST,
                                 _ptr(w), _ptr(Vb), n, ctypes.byref(o),
                                 stream if stream is not None else _stream(torch), ctypes.byref(info))
    _check(st, "qdwhp_eig_noalloc")
    out = (w, Vb.t())
    return out + (info.as_dict(),) if return_info else out


def svd(A, k, opts=None, return_info=False, stream=None):
    """Top-k singular triplets of the m x n float64 CUDA tensor A (QDWHpartial-SVD).

    Returns (U (m,k), S (k,), V (n,k)) [+ info dict]."""
    import torch
    m, n = A.shape
    assert A.dtype == torch.float64 and A.is_cuda
    o = opts if opts is not None else default_opts()
    Acm = A.t().contiguous()
    nbytes = lib().qdwhp_svd_workspace(m, n, k, ctypes.byref(o))
    ws = _workspace(torch, nbytes, A.device)
    Ub = torch.empty((k, m), dtype=torch.float64, device=A.device)
    Vb = torch.empty((k, n), dtype=torch.float64, device=A.device)
    S = torch.empty(k, dtype=torch.float64, device=A.device)
    info = Info()
    st = lib().qdwhp_svd(_ptr(Acm), m, n, m, k, _ptr(Ub), m, _ptr(S), _ptr(Vb), n, _ptr(ws), nbytes,
                         ctypes.byref(o), stream if stream is not None else _stream(torch),
                         ctypes.byref(info))
    _check(st, "qdwhp_svd")
    out = (Ub.t(), S, Vb.t())
    return out + (info.as_dict(),) if return_info else out


def spd_inverse(Z):
    """Inverse of the SPD float64 CUDA matrix Z (a new tensor)."""
    import torch
    n = Z.shape[0]
    Zc = Z.t().contiguous()
    nbytes = lib().qdwhp_spd_inverse_workspace(n)
    ws = _workspace(torch, nbytes, Z.device)
    _check(lib().qdwhp_spd_inverse(_ptr(Zc), n, n, _ptr(ws), nbytes, _stream(torch)), "qdwhp_spd_inverse")
    return Zc.t()


def qr(A, c0=0, q=None):
    """Householder QR of the m x n (m >= n) float64 CUDA tensor A.

    Returns (Qcols, R, tau): Qcols = columns c0 .. c0+q-1 of Q, R the n x n
    triangle."""
    import torch
    m, n = A.shape
    q = n if q is None else q
    Ac = A.t().contiguous()
    tau = torch.empty(n, dtype=torch.float64, device=A.device)
    nbytes = lib().qdwhp_geqrf_workspace(m, n)
    ws = _workspace(torch, nbytes, A.device)
    _check(lib().qdwhp_geqrf(_ptr(Ac), m, n, m, _ptr(tau), _ptr(ws), nbytes, _stream(torch)), "qdwhp_geqrf")
    Qb = torch.empty((max(q, 1), m), dtype=torch.float64, device=A.device)
    _check(lib().qdwhp_orgqr(_ptr(Ac), m, n, m, _ptr(tau), c0, q, _ptr(Qb), m, _ptr(ws), nbytes,
                             _stream(torch)), "qdwhp_orgqr")
    R = torch.triu(Ac.t()[:n, :])
    return Qb.t()[:, :q], R, tau


def syev(H):
    """All eigenpairs of the symmetric float64 CUDA matrix H (block Jacobi):
    (w descending, W, sweeps)."""
    import torch
    n = H.shape[0]
    Hc = H.t().contiguous()
    w = torch.empty(n, dtype=torch.float64, device=H.device)
    Wb = torch.empty((n, n), dtype=torch.float64, device=H.device)
    nbytes = lib().qdwhp_syev_workspace(n)
    ws = _workspace(torch, nbytes, H.device)
    sw = ctypes.c_int(0)
    _check(lib().qdwhp_syev(_ptr(Hc), n, n, _ptr(w), _ptr(Wb), n, _ptr(ws), nbytes, _stream(torch),
                            ctypes.byref(sw)), "qdwhp_syev")
    return w, Wb.t(), sw.value


def eig_hermitian(A, fraction, which="largest", opts=None, return_info=False):
    """Wanted eigenpairs of the complex Hermitian complex128 CUDA tensor A
    (n x n): (w, V[, info]) with w the k real eigenvalues (most wanted first)
    and V (n x k, complex128), each column's largest-magnitude entry real
    positive.  Calls qdwhp_heig."""
    import torch
    n = A.shape[0]
    Ac = A.t().contiguous()                      # column-major, interleaved (re, im)
    k = _count(n, fraction, "qdwhp_heig")
    o = opts if opts is not None else default_opts()
    w = torch.empty(k, dtype=torch.float64, device=A.device)
    Vb = torch.empty((k, n), dtype=torch.complex128, device=A.device)
    nbytes = lib().qdwhp_heig_workspace(n, fraction, ctypes.byref(o))
    ws = _workspace(torch, nbytes, A.device)
    info = Info()
    wh = LARGEST if which == "largest" else SMALLEST
    _check(lib().qdwhp_heig(_ptr(Ac), n, n, fraction, wh, _ptr(w), _ptr(Vb), n, _ptr(ws), nbytes,
                            ctypes.byref(o), _stream(torch), ctypes.byref(info)), "qdwhp_heig")
    V = Vb.t()
    return (w, V, info.as_dict()) if return_info else (w, V)


def zolo_coeffs(l, r):
    """Zolotarev step coefficients computed by the library's host code:
    dict(c=[c_1..c_2r], a=[a_1..a_r], M, l_next)."""
    c = (ctypes.c_double * (2 * r))()
    a = (ctypes.c_double * r)()
    M, ln = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(lib().qdwhp_zolo_coeffs(float(l), int(r), c, a, ctypes.byref(M), ctypes.byref(ln)),
           "qdwhp_zolo_coeffs")
    return dict(c=list(c), a=list(a), M=M.value, l_next=ln.value)


def syev_dc(H):
    """All eigenpairs of the symmetric float64 CUDA matrix H by QDWH-based
    spectral divide and conquer: (w descending, W, recursion depth)."""
    import torch
    n = H.shape[0]
    Hc = H.t().contiguous()
    w = torch.empty(n, dtype=torch.float64, device=H.device)
    Wb = torch.empty((n, n), dtype=torch.float64, device=H.device)
    nbytes = lib().qdwhp_syev_dc_workspace(n)
    ws = _workspace(torch, nbytes, H.device)
    lv = ctypes.c_int(0)
    _check(lib().qdwhp_syev_dc(_ptr(Hc), n, n, _ptr(w), _ptr(Wb), n, _ptr(ws), nbytes, _stream(torch),
                               ctypes.byref(lv)), "qdwhp_syev_dc")
    return w, Wb.t(), lv.value


def gesvj(R):
    """All singular triplets of the square float64 CUDA matrix R (one-sided
    block Jacobi): (U, S descending, V, sweeps)."""
    import torch
    n = R.shape[0]
    Rc = R.t().contiguous()
    S = torch.empty(n, dtype=torch.float64, device=R.device)
    Vb = torch.empty((n, n), dtype=torch.float64, device=R.device)
    nbytes = lib().qdwhp_gesvj_workspace(n)
    ws = _workspace(torch, nbytes, R.device)
    sw = ctypes.c_int(0)
    _check(lib().qdwhp_gesvj(_ptr(Rc), n, n, _ptr(S), _ptr(Vb), n, _ptr(ws), nbytes, _stream(torch),
                             ctypes.byref(sw)), "qdwhp_gesvj")
    return Rc.t(), S, Vb.t(), sw.value


def profile_begin():
    lib().qdwhp_profile_begin()


def profile_end():
    """(algorithmic GEMM flops, summed GEMM kernel ms, launches) since profile_begin."""
    f, t, n = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_int64(0)
    _check(lib().qdwhp_profile_end(ctypes.byref(f), ctypes.byref(t), ctypes.byref(n)), "qdwhp_profile_end")
    return f.value, t.value, n.value


# ---------------------------------------------------------------- batches
def _problem(torch, spec):
    """(Problem, keep-alive list, outputs) for one spec dict:
    {"type": "eig", "A": (n,n) symmetric, "fraction": f, "which": "largest"}
    or {"type": "svd", "A": (m,n), "k": k}."""
    A = spec["A"]
    assert A.dtype == torch.float64 and A.is_cuda
    p = Problem()
    if spec["type"] == "eig":
        n = A.shape[0]
        f = float(spec["fraction"])
        k = min(n, max(1, int(math.floor(f * n + 0.5))))
        Ac = A.contiguous()
        w = torch.empty(k, dtype=torch.float64, device=A.device)
        Vb = torch.empty((k, n), dtype=torch.float64, device=A.device)
        p.type, p.which, p.m, p.n = PROBLEM_EIG, LARGEST if spec.get("which", "largest") == "largest" else SMALLEST, n, n
        p.A, p.lda, p.fraction = Ac.data_ptr(), n, f
        p.w, p.V, p.ldv = w.data_ptr(), Vb.data_ptr(), n
        return p, [Ac, w, Vb], ("eig", w, Vb)
    m, n = A.shape
    k = int(spec["k"])
    Ac = A.t().contiguous()
    S = torch.empty(k, dtype=torch.float64, device=A.device)
    Ub = torch.empty((k, m), dtype=torch.float64, device=A.device)
    Vb = torch.empty((k, n), dtype=torch.float64, device=A.device)
    p.type, p.m, p.n, p.A, p.lda, p.k = PROBLEM_SVD, m, n, Ac.data_ptr(), m, k
    p.w, p.U, p.ldu, p.V, p.ldv = S.data_ptr(), Ub.data_ptr(), m, Vb.data_ptr(), n
    return p, [Ac, S, Ub, Vb], ("svd", S, Ub, Vb)


def _result(out):
    if out[0] == "eig":
        return out[1], out[2].t()
    return out[2].t(), out[1], out[3].t()


def batched(specs, lanes=0, opts=None, return_info=False):
    """Solve a ragged list of problems (see _problem for the spec dicts) with
    qdwhp_batched.  Returns a list of per-problem results ((w, V) for EIG,
    (U, S, V) for SVD) [+ list of info dicts]; raises if any failed."""
    import torch
    o = opts if opts is not None else default_opts()
    count = len(specs)
    probs = (Problem * count)()
    keep, outs = [], []
    for i, sp in enumerate(specs):
        p, kp, out = _problem(torch, sp)
        probs[i] = p
        keep += kp
        outs.append(out)
    dev = specs[0]["A"].device
    nbytes = lib().qdwhp_batched_workspace(count, probs, ctypes.byref(o))
    ws = _workspace(torch, nbytes, dev)
    infos = (Info * count)()
    stat = (ctypes.c_int * count)()
    st = lib().qdwhp_batched(count, probs, _ptr(ws), nbytes, ctypes.byref(o), int(lanes), _stream(torch),
                             infos, stat)
    _check(st, "qdwhp_batched")
    res = [_result(out) for out in outs]
    return (res, [infos[i].as_dict() for i in range(count)]) if return_info else res


def dgemm_grouped(As, Bs, Cs, alphas=None, betas=None, transa=False, transb=False):
    """C_i = alpha_i op(A_i) op(B_i) + beta_i C_i for all i in one launch, on
    column-major buffers (contiguous (cols, rows) tensors, as for dgemm)."""
    import torch
    cnt = len(As)
    alphas = alphas or [1.0] * cnt
    betas = betas or [0.0] * cnt
    M, N, K, LA, LB, LC = [], [], [], [], [], []
    for A, B, C in zip(As, Bs, Cs):
        ka, ma = A.shape
        kb, mb = B.shape
        m, k = (ka, ma) if transa else (ma, ka)
        n = kb if not transb else mb
        M.append(m); N.append(n); K.append(k)
        LA.append(max(1, ma)); LB.append(max(1, mb)); LC.append(max(1, C.shape[1]))
    arr = lambda t, v: (t * cnt)(*v)
    ptrs = lambda ts: (ctypes.c_void_p * cnt)(*[t.data_ptr() for t in ts])
    nbytes = lib().qdwhp_dgemm_grouped_workspace(cnt)
    ws = _workspace(torch, nbytes, As[0].device)
    st = lib().qdwhp_dgemm_grouped(cnt, int(transa), int(transb), arr(ctypes.c_int64, M), arr(ctypes.c_int64, N),
                                   arr(ctypes.c_int64, K), arr(ctypes.c_double, alphas), ptrs(As),
                                   arr(ctypes.c_int64, LA), ptrs(Bs), arr(ctypes.c_int64, LB),
                                   arr(ctypes.c_double, betas), ptrs(Cs), arr(ctypes.c_int64, LC),
                                   _ptr(ws), nbytes, _stream(torch))
    _check(st, "qdwhp_dgemm_grouped")
    return Cs


class Server:
    """Continuous-batching server (qdwhp_serve_*): requests are admitted by
    HBM footprint into a device arena and run concurrently on `lanes`
    streams.  Inputs must not be modified until their request finishes."""

    def __init__(self, arena_bytes, lanes=0, opts=None):
        import torch
        self._torch = torch
        self.opts = opts if opts is not None else default_opts()
        h = ctypes.c_void_p()
        _check(lib().qdwhp_serve_create(int(arena_bytes), int(lanes), ctypes.byref(self.opts), ctypes.byref(h)),
               "qdwhp_serve_create")
        self._h = h
        self._live = {}

    def submit(self, spec):
        """Queue one problem (spec dict as for batched); returns a ticket."""
        torch = self._torch
        p, keep, out = _problem(torch, spec)
        torch.cuda.current_stream().synchronize()   # inputs (and their copies) made on torch's stream are ready
        t = ctypes.c_int64(0)
        _check(lib().qdwhp_serve_submit(self._h, ctypes.byref(p), ctypes.byref(t)), "qdwhp_serve_submit")
        self._live[t.value] = (keep, out)
        return t.value

    def poll(self, ticket, wait=True):
        """None while pending (wait=False); else (result, info dict, latency_ms,
        queue_ms).  Raises if the request failed."""
        info = Info()
        lat, q = ctypes.c_double(0), ctypes.c_double(0)
        st = lib().qdwhp_serve_poll(self._h, int(ticket), int(bool(wait)), ctypes.byref(info),
                                    ctypes.byref(lat), ctypes.byref(q))
        if st == PENDING:
            return None
        keep, out = self._live.pop(ticket)
        _check(st, "qdwhp_serve request")
        return _result(out), info.as_dict(), lat.value, q.value

    def stats(self, reset=False):
        """dict: peak bytes of the arena in use, arena bytes, most requests
        running at once, iteration groups run and the requests they held."""
        pk, cap, pr = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_int(0)
        gr, gq = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().qdwhp_serve_stats(self._h, ctypes.byref(pk), ctypes.byref(cap), ctypes.byref(pr),
                                       ctypes.byref(gr), ctypes.byref(gq), int(bool(reset))), "qdwhp_serve_stats")
        return dict(arena_peak_bytes=pk.value, arena_bytes=cap.value, peak_running=pr.value,
                    groups=gr.value, grouped_requests=gq.value)

    def close(self):
        if self._h:
            _check(lib().qdwhp_serve_destroy(self._h), "qdwhp_serve_destroy")
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
