"""ctypes binding of libdsanls.so (the C ABI declared in include/dsanls.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Device buffers are torch tensors on a ROCm device; their data
pointers and torch's current HIP stream are passed through the ABI.  If the
library is missing, load() raises; there is no fallback implementation.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsanls.so")

SKETCH = {"gaussian": 0, "subsample": 1, "identity": 2, "count": 3, "srht": 4}
SOLVER = {"prox_cd": 0, "pgd": 1}
PRECISION = {"fp32": 0, "bf16": 1}
DENSE, CSR = 0, 1
STATUS = {0: "OK", 1: "INVALID_ARG", 2: "SHAPE", 3: "WORKSPACE", 4: "HIP", 5: "NONFINITE",
          6: "STATE", 7: "UNSUPPORTED", 8: "INTERNAL"}

c_int32, c_int64, c_uint64, c_double, c_vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                              ctypes.c_double, ctypes.c_void_p)
c_size_t, c_float, c_uint32 = ctypes.c_size_t, ctypes.c_float, ctypes.c_uint32


class Config(ctypes.Structure):
    _fields_ = [("m", c_int64), ("n", c_int64), ("k", c_int64), ("d", c_int64),
                ("d_prime", c_int64), ("sketch", c_int32), ("solver", c_int32),
                ("precision", c_int32), ("sweeps", c_int32), ("max_sweeps", c_int32),
                ("clip_upper", c_int32), ("tol", c_double), ("alpha", c_double),
                ("beta", c_double), ("seed", c_uint64), ("warm_hidden", c_int32), ("reserved", c_int32),
                ("row_offset", c_int64), ("col_offset", c_int64), ("m_global", c_int64), ("n_global", c_int64)]


class Matrix(ctypes.Structure):
    _fields_ = [("format", c_int32), ("dense", c_vp), ("ld", c_int64), ("dense_t", c_vp),
                ("ld_t", c_int64), ("rowptr", c_vp), ("colidx", c_vp), ("vals", c_vp),
                ("nnz", c_int64), ("t_rowptr", c_vp), ("t_colidx", c_vp), ("t_vals", c_vp)]


class Stats(ctypes.Structure):
    _fields_ = [("updates", c_int64), ("rows_updated", c_int64), ("sweeps_total", c_int64),
                ("rows_unconverged", c_int64), ("warm_fallbacks", c_int64)]


class Timing(ctypes.Structure):
    _fields_ = [("sketch_ms", c_double), ("product_ms", c_double), ("small_ms", c_double),
                ("nnls_ms", c_double), ("launches", c_int64)]


class DsanlsError(RuntimeError):
    def __init__(self, func, status, message):
        self.status = status
        self.status_name = STATUS.get(status, str(status))
        super().__init__(f"{func}: {self.status_name}: {message}")


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "dsanls_workspace_bytes": (c_int32, [ctypes.POINTER(Config), ctypes.POINTER(Matrix), ctypes.POINTER(c_size_t)]),
    "dsanls_init": (c_int32, [ctypes.POINTER(Config), ctypes.POINTER(Matrix), c_vp, c_vp, c_vp, c_size_t, c_vp,
                              ctypes.POINTER(c_vp)]),
    "dsanls_sketch_update_U": (c_int32, [c_vp, c_int64]),
    "dsanls_sketch_update_V": (c_int32, [c_vp, c_int64]),
    "dsanls_objective": (c_int32, [c_vp, ctypes.POINTER(c_double)]),
    "dsanls_get_stats": (c_int32, [c_vp, ctypes.POINTER(Stats)]),
    "dsanls_debug_fetch": (c_int32, [c_vp, c_int32, c_vp, c_size_t]),
    "dsanls_set_timing": (c_int32, [c_vp, c_int32]),
    "dsanls_get_timing": (c_int32, [c_vp, ctypes.POINTER(Timing)]),
    "dsanls_set_warm_start": (c_int32, [c_vp, c_vp, c_int32, c_int32]),
    "dsanls_set_keep_sketched_rows": (c_int32, [c_vp, c_int32]),
    "dsanls_gather_sketched_rows": (c_int32, [c_vp, c_vp, c_int64, c_vp, c_vp, c_vp, c_int64,
                                              ctypes.POINTER(c_int64)]),
    "dsanls_mlp_param_count": (c_int64, [c_int32, c_int32, c_int32]),
    "dsanls_mlp_workspace_bytes": (c_size_t, [c_int32, c_int32, c_int32, c_int64]),
    "dsanls_mlp_forward": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_vp, c_int64, c_vp, c_vp, c_vp, c_vp,
                                     c_vp, c_vp, c_size_t, c_vp]),
    "dsanls_mlp_gradients": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_vp, c_vp, c_int64, c_vp, c_vp, c_vp,
                                       c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_size_t, c_vp]),
    "dsanls_mlp_train_step": (c_int32, [c_int32, c_int32, c_int32, c_int32, c_vp, c_vp, c_vp, c_vp, c_int64,
                                        c_float, c_int64, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                        c_vp, c_size_t, c_vp]),
    "dsanls_destroy": (c_int32, [c_vp]),
    "dsanls_status_string": (ctypes.c_char_p, [c_int32]),
    "dsanls_last_error": (ctypes.c_char_p, []),
    "dsanls_philox4x32_10": (c_int32, [c_vp, c_vp, c_vp, c_int64, c_vp]),
    "dsanls_gaussian_sketch_t": (c_int32, [c_uint64, c_int64, c_int32, c_int64, c_int64, c_vp, c_int64, c_vp]),
    "dsanls_subsample_workspace_bytes": (c_size_t, [c_int64]),
    "dsanls_subsample_indices": (c_int32, [c_uint64, c_int64, c_int32, c_int64, c_int64, c_vp, c_vp, c_size_t,
                                           c_vp]),
    "dsanls_gemm_workspace_bytes": (c_size_t, [c_int64, c_int64, c_int64]),
    "dsanls_gemm_nt": (c_int32, [c_vp, c_int64, c_vp, c_int64, c_vp, c_int64, c_int64, c_int64, c_int64, c_vp,
                                 c_size_t, c_vp]),
    "dsanls_gemm_nt_bf16": (c_int32, [c_vp, c_int64, c_vp, c_int64, c_vp, c_int64, c_int64, c_int64, c_int64,
                                      c_vp]),
    "dsanls_nnls_workspace_bytes": (c_size_t, [c_int32]),
    "dsanls_nnls_prox_cd": (c_int32, [c_vp, c_vp, c_vp, c_vp, c_int64, c_int32, c_float, c_int32, c_float,
                                      c_int32, c_float, c_vp, c_vp, c_size_t, c_vp]),
    "dsanls_pgd_step": (c_int32, [c_vp, c_vp, c_vp, c_int64, c_int32, c_float, c_float, c_vp, c_size_t, c_vp]),
    "dsanls_nnls_noalloc_scratch_bytes": (c_size_t, []),
    "dsanls_nnls_prox_cd_noalloc": (c_int32, [c_vp, c_vp, c_vp, c_vp, c_int64, c_int32, c_float, c_int32, c_float,
                                              c_int32, c_float, c_vp, c_vp]),
}


def exported_symbols():
    return sorted(_SIGS)


def load(path=LIB_PATH):
    """Load libdsanls.so (built by paper_2009_02845_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2009_02845_amd.build`; "
                           "there is no fallback implementation")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(name, status):
    if status != 0:
        msg = _lib.dsanls_last_error().decode(errors="replace")
        raise DsanlsError(name, status, msg)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_config(m, n, k, d, d_prime=None, sketch="gaussian", solver="prox_cd", precision="fp32",
                sweeps=1, max_sweeps=100, tol=1e-4, alpha=1.0, beta=1.0, clip_upper=False, seed=0,
                warm_hidden=0, row_offset=0, col_offset=0, m_global=0, n_global=0):
    return Config(m=m, n=n, k=k, d=d, d_prime=d if d_prime is None else d_prime,
                  sketch=SKETCH[sketch], solver=SOLVER[solver], precision=PRECISION[precision],
                  sweeps=sweeps, max_sweeps=max_sweeps, clip_upper=int(bool(clip_upper)), tol=tol,
                  alpha=alpha, beta=beta, seed=seed, warm_hidden=warm_hidden, row_offset=row_offset,
                  col_offset=col_offset, m_global=m_global, n_global=n_global)


def dense_matrix(M, Mt=None):
    """Matrix descriptor of a dense row-major device tensor (and optional M^T)."""
    return Matrix(format=DENSE, dense=M.data_ptr(), ld=M.stride(0),
                  dense_t=None if Mt is None else Mt.data_ptr(), ld_t=0 if Mt is None else Mt.stride(0))


def csr_matrix(rowptr, colidx, vals, t_rowptr, t_colidx, t_vals):
    """Matrix descriptor of CSR(M) and CSR(M^T) device tensors."""
    return Matrix(format=CSR, rowptr=rowptr.data_ptr(), colidx=colidx.data_ptr(), vals=vals.data_ptr(),
                  nnz=vals.numel(), t_rowptr=t_rowptr.data_ptr(), t_colidx=t_colidx.data_ptr(),
                  t_vals=t_vals.data_ptr())


def workspace_bytes(cfg, mat):
    lib = load()
    out = c_size_t(0)
    _check("dsanls_workspace_bytes", lib.dsanls_workspace_bytes(ctypes.byref(cfg), ctypes.byref(mat),
                                                                ctypes.byref(out)))
    return out.value


class Solver:
    """One DSANLS context: M (dense or CSR) and the factors U, V on one GPU.

    tensors: dict of the device tensors the descriptor points to (kept alive
    here); U (m x k) and V (n x k) are float32 device tensors updated in
    place by update_U / update_V.
    """

    def __init__(self, cfg, mat, U, V, tensors=(), stream=None):
        import torch
        self.lib = load()
        self.cfg, self.mat = cfg, mat
        self.U, self.V = U, V
        self._keep = list(tensors)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        nbytes = workspace_bytes(cfg, mat)
        # torch's caching allocator returns blocks aligned to >= 512 bytes
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=U.device)
        ctx = c_vp()
        _check("dsanls_init", self.lib.dsanls_init(ctypes.byref(cfg), ctypes.byref(mat), _ptr(U), _ptr(V),
                                                   _ptr(self.workspace), nbytes, _stream(self.stream),
                                                   ctypes.byref(ctx)))
        self.ctx = ctx

    def update_U(self, t):
        _check("dsanls_sketch_update_U", self.lib.dsanls_sketch_update_U(self.ctx, t))

    def update_V(self, t):
        _check("dsanls_sketch_update_V", self.lib.dsanls_sketch_update_V(self.ctx, t))

    def iteration(self, t):
        self.update_U(t)
        self.update_V(t)

    def objective(self):
        out = c_double(0.0)
        _check("dsanls_objective", self.lib.dsanls_objective(self.ctx, ctypes.byref(out)))
        return out.value

    def stats(self):
        s = Stats()
        _check("dsanls_get_stats", self.lib.dsanls_get_stats(self.ctx, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def set_timing(self, enable=True):
        _check("dsanls_set_timing", self.lib.dsanls_set_timing(self.ctx, int(bool(enable))))

    def timing(self):
        """Per-phase GPU milliseconds (HIP events) of the updates timed so far."""
        t = Timing()
        _check("dsanls_get_timing", self.lib.dsanls_get_timing(self.ctx, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in Timing._fields_}

    def fetch(self, which, shape, dtype="float32"):
        """Host copy of an intermediate of the last update (see dsanls_debug_fetch)."""
        import numpy as np
        out = np.empty(shape, dtype=dtype)
        _check("dsanls_debug_fetch", self.lib.dsanls_debug_fetch(self.ctx, which, out.ctypes.data, out.nbytes))
        return out

    def set_warm_start(self, params, hidden, residual=False):
        """Install a packed warm-start network (float32 device tensor), or None."""
        self._warm = params
        _check("dsanls_set_warm_start", self.lib.dsanls_set_warm_start(self.ctx, _ptr(params), hidden,
                                                                        int(bool(residual))))

    def keep_sketched_rows(self, enable=True):
        _check("dsanls_set_keep_sketched_rows", self.lib.dsanls_set_keep_sketched_rows(self.ctx, int(enable)))

    def gather_sketched_rows(self, sel, capacity):
        """Sketched rows a_i of the last update for row indices sel (int32
        device tensor): (rowptr, cols, vals) device tensors."""
        import torch
        n = sel.numel()
        rp = torch.empty(n + 1, dtype=torch.int32, device=sel.device)
        cols = torch.empty(max(capacity, 1), dtype=torch.int32, device=sel.device)
        vals = torch.empty(max(capacity, 1), dtype=torch.float32, device=sel.device)
        nnz = c_int64(0)
        _check("dsanls_gather_sketched_rows", self.lib.dsanls_gather_sketched_rows(
            self.ctx, _ptr(sel), n, _ptr(rp), _ptr(cols), _ptr(vals), capacity, ctypes.byref(nnz)))
        return rp, cols[:nnz.value], vals[:nnz.value]

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.dsanls_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- stand-alone kernels

def philox4x32_10(ctr, key, stream=None):
    """ctr: int32 device tensor (count, 4); key: (count, 2); returns (count, 4) int32 words."""
    import torch
    lib = load()
    out = torch.empty_like(ctr)
    _check("dsanls_philox4x32_10", lib.dsanls_philox4x32_10(_ptr(ctr), _ptr(key), _ptr(out), ctr.shape[0],
                                                            _stream(stream)))
    return out


def gaussian_sketch_t(seed, t, side, n, d, device="cuda", stream=None):
    import torch
    lib = load()
    St = torch.empty((d, n), dtype=torch.float32, device=device)
    _check("dsanls_gaussian_sketch_t", lib.dsanls_gaussian_sketch_t(seed, t, side, n, d, _ptr(St), n,
                                                                    _stream(stream)))
    return St


def subsample_indices(seed, t, side, n, d, device="cuda", stream=None):
    import torch
    lib = load()
    idx = torch.empty(d, dtype=torch.int32, device=device)
    nb = lib.dsanls_subsample_workspace_bytes(n)
    ws = torch.empty(nb, dtype=torch.uint8, device=device)
    _check("dsanls_subsample_indices", lib.dsanls_subsample_indices(seed, t, side, n, d, _ptr(idx), _ptr(ws),
                                                                    nb, _stream(stream)))
    return idx


def gemm_nt(X, Y, out=None, stream=None):
    """C = X Y^T for float32 device tensors X (rows x K), Y (cols x K)."""
    import torch
    lib = load()
    rows, K = X.shape
    cols = Y.shape[0]
    C = out if out is not None else torch.empty((rows, cols), dtype=torch.float32, device=X.device)
    nb = lib.dsanls_gemm_workspace_bytes(rows, cols, K)
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=X.device) if nb else None
    _check("dsanls_gemm_nt", lib.dsanls_gemm_nt(_ptr(X), X.stride(0), _ptr(Y), Y.stride(0), _ptr(C), C.stride(0),
                                                rows, cols, K, _ptr(ws), nb, _stream(stream)))
    return C


def gemm_nt_bf16(X, Y, stream=None):
    """C = X Y^T (FP32) for torch.bfloat16 device tensors X (rows x K), Y (cols x K)."""
    import torch
    lib = load()
    rows, K = X.shape
    cols = Y.shape[0]
    C = torch.empty((rows, cols), dtype=torch.float32, device=X.device)
    _check("dsanls_gemm_nt_bf16", lib.dsanls_gemm_nt_bf16(_ptr(X), X.stride(0), _ptr(Y), Y.stride(0), _ptr(C),
                                                          C.stride(0), rows, cols, K, _stream(stream)))
    return C


def nnls_prox_cd(G, R, C, U, mu, sweeps=1, tol=1e-4, max_sweeps=100, upper=0.0, want_sweeps=False,
                 stream=None):
    """Prox-CD on every row of U (in place).  Returns the per-row sweep counts
    (int32 device tensor) when want_sweeps."""
    import torch
    lib = load()
    rows, k = U.shape
    used = torch.empty(rows, dtype=torch.int32, device=U.device) if want_sweeps else None
    nb = lib.dsanls_nnls_workspace_bytes(k)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=U.device)
    _check("dsanls_nnls_prox_cd", lib.dsanls_nnls_prox_cd(_ptr(G), _ptr(R), _ptr(C), _ptr(U), rows, k, mu,
                                                          sweeps, tol, max_sweeps, upper, _ptr(used),
                                                          _ptr(ws), nb, _stream(stream)))
    return used


def nnls_prox_cd_noalloc(G, R, C, U, mu, sweeps=1, tol=1e-4, max_sweeps=100, upper=0.0, want_sweeps=False,
                         stream=None):
    """nnls_prox_cd through the allocation-free entry point (the library's
    static device scratch instead of a workspace)."""
    import torch
    lib = load()
    rows, k = U.shape
    used = torch.empty(rows, dtype=torch.int32, device=U.device) if want_sweeps else None
    _check("dsanls_nnls_prox_cd_noalloc", lib.dsanls_nnls_prox_cd_noalloc(
        _ptr(G), _ptr(R), _ptr(C), _ptr(U), rows, k, mu, sweeps, tol, max_sweeps, upper, _ptr(used),
        _stream(stream)))
    return used


def pgd_step(G, R, U, mu, upper=0.0, stream=None):
    import torch
    lib = load()
    rows, k = U.shape
    nb = lib.dsanls_nnls_workspace_bytes(k)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=U.device)
    _check("dsanls_pgd_step", lib.dsanls_pgd_step(_ptr(G), _ptr(R), _ptr(U), rows, k, mu, upper, _ptr(ws), nb,
                                                  _stream(stream)))


# ----------------------------------------------------------------- warm-start network

def mlp_param_count(d, k, hidden):
    return load().dsanls_mlp_param_count(d, k, hidden)


def mlp_pack(p, device="cuda"):
    """Pack a dict of numpy weights (W1a, W1u, b1, W2, b2) into the flat layout."""
    import numpy as np
    import torch
    flat = np.concatenate([np.ascontiguousarray(p[n], dtype=np.float32).ravel()
                           for n in ("W1a", "W1u", "b1", "W2", "b2")])
    return torch.from_numpy(flat).to(device)


def mlp_unpack(flat, d, k, hidden):
    """Inverse of mlp_pack (host numpy float64 arrays)."""
    import numpy as np
    x = flat.detach().cpu().numpy().astype(np.float64) if hasattr(flat, "detach") else np.asarray(flat)
    out, o = {}, 0
    for name, shape in (("W1a", (d, hidden)), ("W1u", (hidden, k)), ("b1", (hidden,)), ("W2", (k, hidden)),
                        ("b2", (k,))):
        n = int(np.prod(shape))
        out[name] = x[o:o + n].reshape(shape)
        o += n
    return out


class MLP:
    """Device-side warm-start network: forward, gradients and Adam steps."""

    def __init__(self, d, k, hidden, params, max_rows, stream=None, residual=False):
        import torch
        self.lib = load()
        self.d, self.k, self.h = d, k, hidden
        self.residual = int(bool(residual))
        self.params = params
        self.grads = torch.zeros_like(params)
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.step = 0
        self.loss = torch.zeros(4, dtype=torch.float32, device=params.device)
        self.ws_bytes = self.lib.dsanls_mlp_workspace_bytes(d, k, hidden, max_rows)
        self.ws = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=params.device)
        self.max_rows = max_rows
        self.stream = stream

    def forward(self, a_rowptr, a_cols, a_vals, U):
        import torch
        rows = U.shape[0]
        out = torch.empty((rows, self.k), dtype=torch.float32, device=U.device)
        _check("dsanls_mlp_forward", self.lib.dsanls_mlp_forward(
            self.d, self.k, self.h, self.residual, _ptr(self.params), rows, _ptr(a_rowptr), _ptr(a_cols), _ptr(a_vals),
            _ptr(U), _ptr(out), _ptr(self.ws), self.ws_bytes, _stream(self.stream)))
        return out

    def gradients(self, batch):
        a_rp, a_c, a_v, c_cp, c_r, c_v, U, Y = batch
        _check("dsanls_mlp_gradients", self.lib.dsanls_mlp_gradients(
            self.d, self.k, self.h, self.residual, _ptr(self.params), _ptr(self.grads), U.shape[0], _ptr(a_rp), _ptr(a_c),
            _ptr(a_v), _ptr(c_cp), _ptr(c_r), _ptr(c_v), _ptr(U), _ptr(Y), _ptr(self.loss), _ptr(self.ws),
            self.ws_bytes, _stream(self.stream)))
        return self.grads

    def train_step(self, batch, lr):
        a_rp, a_c, a_v, c_cp, c_r, c_v, U, Y = batch
        self.step += 1
        _check("dsanls_mlp_train_step", self.lib.dsanls_mlp_train_step(
            self.d, self.k, self.h, self.residual, _ptr(self.params), _ptr(self.grads), _ptr(self.m), _ptr(self.v), self.step,
            lr, U.shape[0], _ptr(a_rp), _ptr(a_c), _ptr(a_v), _ptr(c_cp), _ptr(c_r), _ptr(c_v), _ptr(U), _ptr(Y),
            _ptr(self.loss), _ptr(self.ws), self.ws_bytes, _stream(self.stream)))

    def last_loss(self):
        return float(self.loss[0].item()) + float(self.loss[1].item())
