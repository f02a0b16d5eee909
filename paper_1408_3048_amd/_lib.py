"""ctypes binding of libmm.so (include/mm.h): argument marshalling only.

Every function here forwards to the C entry point of the same name; all
arithmetic runs in the library's HIP kernels.  Torch tensors supply device
memory and the current HIP stream.  If the library is missing this module
raises instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmm.so")

MM_OK, MM_ERR_ARG, MM_ERR_DEVICE, MM_ERR_RANK = 0, -1, -2, -3
MM_ERR_NOT_SPD, MM_ERR_BREAKDOWN, MM_ERR_NOCONV, MM_ERR_STATE = -4, -5, -6, -7
MM_F32, MM_F64 = 0, 1
MM_WIN_GAUSS, MM_WIN_GAUSS2, MM_WIN_RECT = 0, 1, 2
MM_FP64, MM_MIXED, MM_MIXED_IR = 0, 1, 2
MM_COARSE_NONE, MM_COARSE_ZS = 0, 1
MM_BJ, MM_2LVL, MM_ADEF2 = 0, 1, 2
_PRECOND = {"bj": MM_BJ, "2lvl": MM_2LVL, "adef2": MM_ADEF2}

STATUS_NAMES = {0: "MM_OK", -1: "MM_ERR_ARG", -2: "MM_ERR_DEVICE", -3: "MM_ERR_RANK",
                -4: "MM_ERR_NOT_SPD", -5: "MM_ERR_BREAKDOWN", -6: "MM_ERR_NOCONV",
                -7: "MM_ERR_STATE"}

EXPORTED = [
    "mm_default_opts", "mm_plan", "mm_destroy", "mm_n_obs", "mm_n_stokes", "mm_obs_pixels",
    "mm_hits", "mm_sorted_samples", "mm_interval_taps", "mm_coarse_rank", "mm_coarse_columns",
    "mm_coarse_matrix", "mm_apply_P", "mm_apply_Ninv", "mm_apply_PT", "mm_rhs", "mm_apply_A",
    "mm_precond_bj", "mm_precond_2lvl", "mm_pcg_solve", "mm_plan_time_ms", "mm_gemm_tn_f64",
    "mm_profile", "mm_profile_read", "mm_last_error", "mm_plan_batched", "mm_n_problems",
    "mm_problem_pixels", "mm_coarse_problem_columns", "mm_fft_lengths", "mm_lag_correlations",
    "mm_tap_derivatives", "mm_adjoint", "mm_coarse_from_krylov", "mm_lanczos_ritz",
    "mm_coarse_kind", "mm_coarse_ritz_values", "mm_coarse_dense_columns", "mm_precond_adef2",
    "mm_gemm_tn_f64_noalloc", "mm_pt_range",
]


class MMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class mm_psd(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_double), ("f_knee", ctypes.c_double), ("alpha", ctypes.c_double)]


class mm_opts(ctypes.Structure):
    _fields_ = [("n_stokes", ctypes.c_int), ("lambda_", ctypes.c_int), ("f_samp", ctypes.c_double),
                ("window", ctypes.c_int), ("precision", ctypes.c_int), ("coarse", ctypes.c_int),
                ("rank_tol", ctypes.c_double), ("rcond_min", ctypes.c_double),
                ("fft_len_f64", ctypes.c_int), ("fft_len_f32", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("graph", ctypes.c_int), ("autotune", ctypes.c_int),
                ("az_fp16", ctypes.c_int), ("pt_range", ctypes.c_int)]


class mm_solve_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("outer_iterations", ctypes.c_int),
                ("replacements", ctypes.c_int), ("status", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int),
                ("history_len", ctypes.c_int)]


_lib = None


def load():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1408_3048_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I32, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "mm_default_opts": (None, [ctypes.POINTER(mm_opts)]),
        "mm_plan": (I, [ctypes.POINTER(P), I64, P, P, I, I64, I32, P, P, ctypes.POINTER(mm_opts)]),
        "mm_destroy": (None, [P]),
        "mm_n_obs": (I64, [P]),
        "mm_n_stokes": (I, [P]),
        "mm_obs_pixels": (I, [P, P]),
        "mm_hits": (I, [P, P]),
        "mm_sorted_samples": (I, [P, P]),
        "mm_interval_taps": (I, [P, I32, P, I]),
        "mm_coarse_rank": (I, [P]),
        "mm_coarse_columns": (I, [P, P, I]),
        "mm_coarse_matrix": (I, [P, P, I64]),
        "mm_apply_P": (I, [P, P, P, I]),
        "mm_apply_Ninv": (I, [P, P, P, I]),
        "mm_apply_PT": (I, [P, P, I, P]),
        "mm_rhs": (I, [P, P, I, P]),
        "mm_apply_A": (I, [P, P, P, I]),
        "mm_precond_bj": (I, [P, P, P]),
        "mm_precond_2lvl": (I, [P, P, P]),
        "mm_precond_adef2": (I, [P, P, P]),
        "mm_pcg_solve": (I, [P, P, P, I, I, D, I, ctypes.POINTER(mm_solve_info)]),
        "mm_plan_time_ms": (D, [P]),
        "mm_gemm_tn_f64": (I, [P, P, P, I64, I32, I32, P]),
        "mm_gemm_tn_f64_noalloc": (I, [P, P, P, I64, I32, I32, P]),
        "mm_pt_range": (I, [P]),
        "mm_profile": (I, [P, I]),
        "mm_profile_read": (I, [P, I, ctypes.POINTER(I64), ctypes.POINTER(D)]),
        "mm_last_error": (ctypes.c_char_p, []),
        "mm_plan_batched": (I, [ctypes.POINTER(P), I32, P, I64, P, P, I, I64, I32, P, P,
                                ctypes.POINTER(mm_opts)]),
        "mm_n_problems": (I, [P]),
        "mm_problem_pixels": (I, [P, P]),
        "mm_coarse_problem_columns": (I, [P, P, I]),
        "mm_fft_lengths": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "mm_lag_correlations": (I, [P, P, P, P]),
        "mm_tap_derivatives": (I, [P, P, I64]),
        "mm_adjoint": (I, [P, P, P, P, I, I, I, D, I, P, P, I, P, ctypes.POINTER(mm_solve_info)]),
        "mm_coarse_from_krylov": (I, [P, P, P, D, I, I, D, I, ctypes.POINTER(mm_solve_info)]),
        "mm_lanczos_ritz": (I, [P, P, I, D, I, P, P]),
        "mm_coarse_kind": (I, [P]),
        "mm_coarse_ritz_values": (I, [P, P, I]),
        "mm_coarse_dense_columns": (I64, [P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error():
    return load().mm_last_error().decode()


def check(status):
    if status != MM_OK:
        raise MMError(status, last_error())
    return status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _validate(*specs):
    """Raise before any library call unless every (tensor, name, dtypes, numel) in specs is
    a contiguous tensor of one of dtypes with numel elements (None: any) on a GPU: the
    library dereferences the raw pointers in its kernels, so a host tensor, a wrong element
    type or a short buffer would be read or written out of bounds on the device.  Types,
    lengths and layouts of every argument are checked before their devices."""
    import torch
    for t, name, dtypes, numel in specs:
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
        if t.dtype not in dtypes:
            raise TypeError(f"{name}: dtype {t.dtype} not in {tuple(str(d) for d in dtypes)}")
        if numel is not None and t.numel() != numel:
            raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: tensor must be contiguous")
    for t, name, _, _ in specs:
        if not t.is_cuda:
            raise ValueError(f"{name}: tensor must be on the GPU (got device {t.device})")


def _check(t, name, dtypes, numel=None):
    _validate((t, name, dtypes, numel))
    return t


def _f64():
    import torch
    return (torch.float64,)


def _f32_or_f64():
    import torch
    return (torch.float32, torch.float64)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# --------------------------------------------------------------------------- wrappers

class Plan:
    """Owns an mm_plan_t.  Inputs are torch CUDA tensors (pix int32 [N],
    weights float32/float64 [N, 2] or None) and host arrays (offsets int64 [K+1],
    psd float64 [K, 3] = (sigma, f_knee, alpha)).  problem_intervals (int32
    [B+1]) makes a batched plan of B independent problems (mm_plan_batched)."""

    def __init__(self, pix, weights, n_pix, offsets, psd, *, n_stokes=3, lam=1024, f_samp=200.0,
                 window="gauss", precision="fp64", coarse=False, rank_tol=1e-10, rcond_min=1e-8,
                 fft_len_f64=0, fft_len_f32=0, problem_intervals=None, graph=True,
                 autotune=False, az_fp16=True, pt_range=0):
        import torch
        self._h = ctypes.c_void_p()
        if not isinstance(pix, torch.Tensor) or pix.dim() != 1:
            raise ValueError("pix: expected a 1-D tensor")
        specs = [(pix, "pix", (torch.int32,), None)]
        wdt = MM_F64
        if weights is not None:
            specs.append((weights, "weights", _f32_or_f64(), 2 * pix.shape[0]))
            if isinstance(weights, torch.Tensor) and tuple(weights.shape) != (pix.shape[0], 2):
                raise ValueError(f"weights: shape {tuple(weights.shape)}, expected "
                                 f"({pix.shape[0]}, 2)")
        elif n_stokes != 1:
            raise ValueError("weights: required for n_stokes = 3")
        _validate(*specs)
        if weights is not None:
            wdt = MM_F64 if weights.dtype == torch.float64 else MM_F32
        L = load()
        self._lib = L
        opts = mm_opts()
        L.mm_default_opts(ctypes.byref(opts))
        opts.n_stokes = n_stokes
        opts.lambda_ = int(lam)
        opts.f_samp = float(f_samp)
        opts.window = {"gauss": MM_WIN_GAUSS, "gauss2": MM_WIN_GAUSS2, "rect": MM_WIN_RECT}[window]
        opts.precision = {"fp64": MM_FP64, "mixed": MM_MIXED}[precision]
        opts.coarse = MM_COARSE_ZS if coarse else MM_COARSE_NONE
        opts.rank_tol = float(rank_tol)
        opts.rcond_min = float(rcond_min)
        opts.fft_len_f64 = int(fft_len_f64)
        opts.fft_len_f32 = int(fft_len_f32)
        opts.stream = _stream()
        opts.graph = 1 if graph else 0
        opts.autotune = 1 if autotune else 0
        opts.az_fp16 = 1 if az_fp16 else 0
        opts.pt_range = int(pt_range)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        ps = np.ascontiguousarray(psd, dtype=np.float64).reshape(-1, 3)
        self.n_samples = int(pix.shape[0])
        self.n_intervals = int(off.shape[0] - 1)
        self.n_stokes = n_stokes
        self.precision = precision
        if problem_intervals is None:
            st = L.mm_plan(ctypes.byref(self._h), self.n_samples, _ptr(pix), _ptr(weights), wdt,
                           int(n_pix), self.n_intervals, off.ctypes.data_as(ctypes.c_void_p),
                           ps.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts))
        else:
            pint = np.ascontiguousarray(problem_intervals, dtype=np.int32)
            st = L.mm_plan_batched(ctypes.byref(self._h), int(pint.shape[0] - 1),
                                   pint.ctypes.data_as(ctypes.c_void_p), self.n_samples,
                                   _ptr(pix), _ptr(weights), wdt, int(n_pix), self.n_intervals,
                                   off.ctypes.data_as(ctypes.c_void_p),
                                   ps.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opts))
        check(st)
        self.n_obs = int(L.mm_n_obs(self._h))
        self.n_vec = self.n_obs * n_stokes
        self.n_problems = int(L.mm_n_problems(self._h))
        self.lam = int(lam)
        self.plan_ms = float(L.mm_plan_time_ms(self._h))

    @classmethod
    def from_scan(cls, scan, device="cuda", weights_dtype=None, **kw):
        import torch
        pix = torch.from_numpy(np.ascontiguousarray(scan.pix, dtype=np.int32)).to(device)
        w = None
        if scan.weights is not None:
            w = torch.from_numpy(np.ascontiguousarray(scan.weights)).to(device)
            if weights_dtype is not None:
                w = w.to(weights_dtype)
        psd = np.stack([scan.sigma, scan.fknee, scan.alpha], axis=1)
        kw.setdefault("lam", scan.lam)
        kw.setdefault("f_samp", scan.f_samp)
        if getattr(scan, "problem_offsets", None) is not None:
            kw.setdefault("problem_intervals", scan.problem_offsets)
        return cls(pix, w, scan.n_pix, scan.offsets, psd, n_stokes=scan.n_stokes, **kw)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.mm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # ---- queries
    def obs_pixels(self):
        import torch
        out = torch.empty(self.n_obs, dtype=torch.int32, device="cuda")
        check(self._lib.mm_obs_pixels(self._h, _ptr(out)))
        return out

    def hits(self):
        import torch
        out = torch.empty(self.n_obs, dtype=torch.int32, device="cuda")
        check(self._lib.mm_hits(self._h, _ptr(out)))
        return out

    def sorted_samples(self):
        import torch
        out = torch.empty(self.n_samples, dtype=torch.int32, device="cuda")
        check(self._lib.mm_sorted_samples(self._h, _ptr(out)))
        return out

    def interval_taps(self, j):
        n = self._lib.mm_interval_taps(self._h, int(j), None, 0)
        check(min(n, 0))
        out = np.empty(n, dtype=np.float64)
        self._lib.mm_interval_taps(self._h, int(j), out.ctypes.data_as(ctypes.c_void_p), n)
        return out

    def coarse_rank(self):
        r = self._lib.mm_coarse_rank(self._h)
        check(min(r, 0))
        return r

    def coarse_columns(self):
        r = self.coarse_rank()
        out = np.empty(r, dtype=np.int32)
        self._lib.mm_coarse_columns(self._h, out.ctypes.data_as(ctypes.c_void_p), r)
        return out

    def fft_lengths(self):
        """(n_r of the FP64 operator, n_r of the FP32 operator or 0)."""
        a, b = ctypes.c_int(), ctypes.c_int()
        check(self._lib.mm_fft_lengths(self._h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def pt_range(self):
        """Samples per P^T work range of the plan."""
        v = self._lib.mm_pt_range(self._h)
        check(min(v, 0))
        return v

    def problem_pixels(self):
        """Host int64 [B+1]: first compact pixel of every problem."""
        out = np.empty(self.n_problems + 1, dtype=np.int64)
        check(self._lib.mm_problem_pixels(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def coarse_problem_columns(self):
        out = np.empty(self.n_problems + 1, dtype=np.int32)
        r = self._lib.mm_coarse_problem_columns(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                                self.n_problems + 1)
        check(min(r, 0))
        return out

    def coarse_matrix(self):
        """E restricted to the kept columns (r_eff x r_eff); for a batched plan the list of
        per-problem diagonal blocks."""
        r = self.coarse_rank()
        if self.n_problems == 1:
            out = np.empty((r, r), dtype=np.float64)
            self._lib.mm_coarse_matrix(self._h, out.ctypes.data_as(ctypes.c_void_p), r * r)
            return out
        co = self.coarse_problem_columns()
        sizes = np.diff(co)
        flat = np.empty(int((sizes.astype(np.int64) ** 2).sum()), dtype=np.float64)
        self._lib.mm_coarse_matrix(self._h, flat.ctypes.data_as(ctypes.c_void_p), flat.shape[0])
        out, o = [], 0
        for k in sizes:
            out.append(flat[o:o + k * k].reshape(k, k))
            o += k * k
        return out

    # ---- kernel timing (HIP events on the plan's stream)
    KERNELS = {"ninv32": 0, "ninv64": 1, "pt32": 2, "pt64": 3, "precond": 4, "vec": 5}

    def profile(self, enable=True):
        check(self._lib.mm_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        out = {}
        for name, k in self.KERNELS.items():
            n = ctypes.c_int64()
            t = ctypes.c_double()
            check(self._lib.mm_profile_read(self._h, k, ctypes.byref(n), ctypes.byref(t)))
            out[name] = (int(n.value), float(t.value))
        return out

    # ---- operators
    def _vec(self):
        import torch
        return torch.empty(self.n_vec, dtype=torch.float64, device="cuda")

    def _map(self, t, name):
        return (t, name, _f64(), self.n_vec)

    def _tod(self, t, name, dtypes=None):
        return (t, name, dtypes or _f32_or_f64(), self.n_samples)

    def apply_P(self, x, dtype=None):
        import torch
        dtype = dtype or torch.float64
        _validate(self._map(x, "x"))
        if dtype not in _f32_or_f64():
            raise TypeError(f"dtype {dtype} not in (torch.float32, torch.float64)")
        y = torch.empty(self.n_samples, dtype=dtype, device="cuda")
        check(self._lib.mm_apply_P(self._h, _ptr(x), _ptr(y),
                                   MM_F64 if dtype == torch.float64 else MM_F32))
        return y

    def apply_Ninv(self, y, precision="fp64"):
        import torch
        p = MM_FP64 if precision == "fp64" else MM_MIXED
        want = torch.float64 if p == MM_FP64 else torch.float32
        _validate(self._tod(y, "y", (want,)))
        z = torch.empty_like(y)
        check(self._lib.mm_apply_Ninv(self._h, _ptr(y), _ptr(z), p))
        return z

    def apply_PT(self, z):
        import torch
        _validate(self._tod(z, "z"))
        x = self._vec()
        check(self._lib.mm_apply_PT(self._h, _ptr(z), MM_F64 if z.dtype == torch.float64 else MM_F32,
                                    _ptr(x)))
        return x

    def rhs(self, d):
        import torch
        _validate(self._tod(d, "d"))
        b = self._vec()
        check(self._lib.mm_rhs(self._h, _ptr(d), MM_F64 if d.dtype == torch.float64 else MM_F32,
                               _ptr(b)))
        return b

    def apply_A(self, x, precision="fp64", out=None):
        _validate(self._map(x, "x"), *([self._map(out, "out")] if out is not None else []))
        if out is not None:
            if out.data_ptr() == x.data_ptr():
                raise ValueError("apply_A: x and out may not alias")
        y = self._vec() if out is None else out
        check(self._lib.mm_apply_A(self._h, _ptr(x), _ptr(y),
                                   MM_FP64 if precision == "fp64" else MM_MIXED))
        return y

    def precond_bj(self, r):
        _validate(self._map(r, "r"))
        z = self._vec()
        check(self._lib.mm_precond_bj(self._h, _ptr(r), _ptr(z)))
        return z

    def precond_2lvl(self, r):
        _validate(self._map(r, "r"))
        z = self._vec()
        check(self._lib.mm_precond_2lvl(self._h, _ptr(r), _ptr(z)))
        return z

    def precond_adef2(self, r):
        _validate(self._map(r, "r"))
        z = self._vec()
        check(self._lib.mm_precond_adef2(self._h, _ptr(r), _ptr(z)))
        return z

    # ---- adjoint
    def lag_correlations(self, u, v):
        """c[j, k], k = 0..lambda: lag cross-correlations of FP64 TOD u, v per interval."""
        import torch
        _validate(self._tod(u, "u", _f64()), self._tod(v, "v", _f64()))
        c = torch.empty((self.n_intervals, self.lam + 1), dtype=torch.float64, device="cuda")
        check(self._lib.mm_lag_correlations(self._h, _ptr(u), _ptr(v), _ptr(c)))
        return c

    def tap_derivatives(self):
        """dt[j, i, k]: derivatives of interval j's taps w.r.t. (sigma, f_knee, alpha)[i]."""
        out = np.zeros((self.n_intervals, 3, self.lam + 1), dtype=np.float64)
        check(self._lib.mm_tap_derivatives(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                           out.size))
        return out

    def adjoint(self, m_hat, g, d, precond="bj", precision="fp64", tol=1e-10, max_iter=3000,
                grad_d_dtype=None, want_psd=True):
        """(dL/dd, dL/dpsd [K, 3] numpy, mu, info) for g = dL/dm_hat."""
        import torch
        _validate(self._map(m_hat, "m_hat"), self._map(g, "g"), self._tod(d, "d"))
        grad_d_dtype = grad_d_dtype or d.dtype
        if grad_d_dtype not in _f32_or_f64():
            raise TypeError(f"grad_d_dtype {grad_d_dtype} not in (torch.float32, torch.float64)")
        gd = torch.empty(self.n_samples, dtype=grad_d_dtype, device="cuda")
        gp = np.zeros((self.n_intervals, 3), dtype=np.float64)
        mu = torch.empty(self.n_vec, dtype=torch.float64, device="cuda")
        infos = (mm_solve_info * self.n_problems)()
        st = self._lib.mm_adjoint(
            self._h, _ptr(m_hat), _ptr(g), _ptr(d), MM_F64 if d.dtype == torch.float64 else MM_F32,
            _PRECOND[precond],
            {"fp64": MM_FP64, "mixed": MM_MIXED, "mixed_ir": MM_MIXED_IR}[precision], float(tol),
            int(max_iter), _ptr(mu), _ptr(gd),
            MM_F64 if grad_d_dtype == torch.float64 else MM_F32,
            gp.ctypes.data_as(ctypes.c_void_p) if want_psd else None, infos)
        check(st)
        info = dict(iterations=infos[0].iterations, rel_residual=infos[0].rel_residual,
                    solve_ms=infos[0].solve_ms)
        return gd, gp, mu, info

    def _infos(self, max_iter, history):
        B = self.n_problems
        infos = (mm_solve_info * B)()
        hists = []
        for i in range(B):
            h = np.zeros(max_iter + 8 if history else 1, dtype=np.float64)
            hists.append(h)
            if history:
                infos[i].history = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
                infos[i].history_cap = h.shape[0]
        return infos, hists

    def pcg_solve(self, b, x0=None, precond="bj", precision="fp64", tol=1e-8, max_iter=1000,
                  history=True, raise_on_error=True):
        """Returns (x, info dict); for a batched plan info["problems"] lists the info of
        every problem and the top-level fields are those of problem 0 plus totals."""
        import torch
        _validate(self._map(b, "b"), *([self._map(x0, "x0")] if x0 is not None else []))
        x = torch.zeros_like(b) if x0 is None else x0.clone()
        infos, hists = self._infos(max_iter, history)
        st = self._lib.mm_pcg_solve(self._h, _ptr(b), _ptr(x),
                                    _PRECOND[precond],
                                    {"fp64": MM_FP64, "mixed": MM_MIXED,
                                     "mixed_ir": MM_MIXED_IR}[precision],
                                    float(tol), int(max_iter), infos)
        return x, self._info_dict(st, infos, hists, raise_on_error)

    def _info_dict(self, st, infos, hists, raise_on_error):
        B = self.n_problems
        per = [dict(status=infos[i].status, iterations=infos[i].iterations,
                    outer_iterations=infos[i].outer_iterations,
                    replacements=infos[i].replacements, rel_residual=infos[i].rel_residual,
                    solve_ms=infos[i].solve_ms, history=hists[i][:infos[i].history_len].copy())
               for i in range(B)]
        out = dict(per[0])
        out["status"] = st
        if B > 1:
            out["problems"] = per
            out["iterations_max"] = max(p["iterations"] for p in per)
            out["iterations_sum"] = sum(p["iterations"] for p in per)
            out["rel_residual_max"] = max(p["rel_residual"] for p in per)
        if raise_on_error and st != MM_OK:
            raise MMError(st, last_error())
        return out

    # ---- a posteriori coarse space
    def coarse_from_krylov(self, b, tol=1e-8, max_iter=1000, krylov_dim=0, eps_tol=0.2,
                           max_cols=0, history=True, raise_on_error=True):
        """Block-Jacobi FP64 PCG solve of A x = b that records its Krylov process and
        replaces the plan's coarse space with Z_D (Ritz vectors of M_BD A with Ritz value
        below eps_tol).  Returns (x, info dict) like pcg_solve."""
        import torch
        _validate(self._map(b, "b"))
        x = torch.zeros_like(b)
        infos, hists = self._infos(max_iter, history)
        st = self._lib.mm_coarse_from_krylov(self._h, _ptr(b), _ptr(x), float(tol),
                                             int(max_iter), int(krylov_dim), float(eps_tol),
                                             int(max_cols), infos)
        return x, self._info_dict(st, infos, hists, raise_on_error)

    def coarse_kind(self):
        """0: none, 1: Z_S, 2: Z_D."""
        k = self._lib.mm_coarse_kind(self._h)
        check(min(k, 0))
        return k

    def ritz_values(self):
        """Ritz value of every kept Z_D column (host FP64 [r_eff])."""
        r = self.coarse_rank()
        out = np.empty(r, dtype=np.float64)
        check(min(self._lib.mm_coarse_ritz_values(self._h, out.ctypes.data_as(ctypes.c_void_p),
                                                  r), 0))
        return out

    def dense_columns(self):
        """The kept Z_D columns: list over problems of CUDA FP64 [r_b, n_stokes * pixels_b]."""
        import torch
        n = self._lib.mm_coarse_dense_columns(self._h, None)
        check(min(n, 0))
        flat = torch.empty(max(int(n), 1), dtype=torch.float64, device="cuda")
        check(min(self._lib.mm_coarse_dense_columns(self._h, _ptr(flat)), 0))
        co = self.coarse_problem_columns()
        pp = self.problem_pixels()
        out, o = [], 0
        for b in range(self.n_problems):
            r, nb = int(co[b + 1] - co[b]), int(pp[b + 1] - pp[b]) * self.n_stokes
            out.append(flat[o:o + r * nb].reshape(r, nb))
            o += r * nb
        return out


def lanczos_ritz(alpha, rz, eps_tol=0.2, max_cols=None):
    """Host helper of the Z_D construction: (theta [r], S [m, r]) of the Lanczos matrix of
    m PCG steps with step lengths alpha[0..m) and r^T z products rz[0..m), Ritz values
    below eps_tol."""
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    rz = np.ascontiguousarray(rz, dtype=np.float64)
    m = alpha.shape[0]
    cap = int(max_cols) if max_cols else m
    theta = np.empty(cap, dtype=np.float64)
    S = np.empty(m * cap, dtype=np.float64)
    r = load().mm_lanczos_ritz(alpha.ctypes.data_as(ctypes.c_void_p),
                               rz.ctypes.data_as(ctypes.c_void_p), m, float(eps_tol), cap,
                               theta.ctypes.data_as(ctypes.c_void_p),
                               S.ctypes.data_as(ctypes.c_void_p))
    check(min(r, 0))
    return theta[:r].copy(), S[:m * r].reshape(m, r).copy()


def _validate_gemm(A, B):
    import torch
    if (not isinstance(A, torch.Tensor) or not isinstance(B, torch.Tensor) or A.dim() != 2
            or B.dim() != 2 or A.shape[0] != B.shape[0]):
        raise ValueError("A and B: expected 2-D tensors [n, ra] and [n, rb]")
    _validate((A, "A", _f64(), None), (B, "B", _f64(), None))


def gemm_tn_f64(A, B):
    """C = A^T B (FP64 matrix cores) for CUDA row-major A [n, ra], B [n, rb]."""
    import torch
    _validate_gemm(A, B)
    C = torch.empty((A.shape[1], B.shape[1]), dtype=torch.float64, device="cuda")
    check(load().mm_gemm_tn_f64(_stream(), _ptr(A), _ptr(B), A.shape[0], A.shape[1], B.shape[1],
                                _ptr(C)))
    return C


def gemm_tn_f64_noalloc(A, B, C):
    """C = A^T B like gemm_tn_f64 through the allocation-free entry point: C is a
    caller-owned CUDA FP64 [ra, rb] tensor; the work is enqueued on the current stream."""
    _validate_gemm(A, B)
    _validate((C, "C", _f64(), A.shape[1] * B.shape[1]))
    check(load().mm_gemm_tn_f64_noalloc(_stream(), _ptr(A), _ptr(B), A.shape[0], A.shape[1],
                                        B.shape[1], _ptr(C)))
    return C
