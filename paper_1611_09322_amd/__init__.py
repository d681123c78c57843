"""Python binding of the gfx950 PSE Brownian sampler (libpse.so).

Argument marshalling only: every step of the sampler runs in the HIP library.
The functions named pse_* mirror the C ABI declared in include/pse.h one to
one; `Sampler` is a small convenience wrapper over them.  Device memory and
the stream come from PyTorch (ROCm build): tensors must live on a HIP device
with the element type of the context's precision (float64 for "fp64",
float32 for "fp32" and "mixed").  There is no CPU fallback: without the built
library every call raises.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpse.so")

PSE_OK = 0
PSE_ERR_NOT_CONVERGED = -6
PSE_WARN_PRECOND_FALLBACK = 1
MLP_NPARAM = 7312
PRECISION = {"fp64": 0, "fp32": 1, "mixed": 2}
FLAG_NOISE_KSPACE = 1
FLAG_FULL_LANCZOS = 2


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("box", ctypes.c_double),
        ("a", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("kT", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("rcut", ctypes.c_double),
        ("grid", ctypes.c_int32),
        ("support", ctypes.c_int32),
        ("gauss_m", ctypes.c_double),
        ("lanczos_tol", ctypes.c_double),
        ("lanczos_max_iter", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("precond", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("tol", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [
        ("lanczos_iters", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("lanczos_rel_change", ctypes.c_double),
        ("max_neighbors", ctypes.c_int32),
        ("precond_fallbacks", ctypes.c_int32),
        ("neighbor_pairs", ctypes.c_int64),
        ("nbr_index_bytes", ctypes.c_int32),
        ("lds_block_edge", ctypes.c_int32),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Derived(ctypes.Structure):
    _fields_ = [
        ("h", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("gauss_m", ctypes.c_double),
        ("eta_se", ctypes.c_double),
        ("eps_real", ctypes.c_double),
        ("eps_wave", ctypes.c_double),
        ("eps_quad", ctypes.c_double),
        ("cells", ctypes.c_int32),
        ("self_real", ctypes.c_double),
        ("eps_alias", ctypes.c_double),
        ("eps_real_tail", ctypes.c_double),
        ("eps_real_coherent", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [
        ("tol", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("n_iter", ctypes.c_double),
        ("c_pair", ctypes.c_double),
        ("c_node", ctypes.c_double),
        ("c_fft", ctypes.c_double),
        ("c_particle", ctypes.c_double),
        ("max_grid", ctypes.c_int32),
        ("with_forces", ctypes.c_int32),
        ("deterministic", ctypes.c_int32),
    ]


class TuningInfo(ctypes.Structure):
    _fields_ = [
        ("model_seconds", ctypes.c_double),
        ("eps_real", ctypes.c_double),
        ("eps_wave", ctypes.c_double),
        ("eps_quad", ctypes.c_double),
        ("eps_alias", ctypes.c_double),
        ("pairs_per_particle", ctypes.c_double),
        ("xi_star", ctypes.c_double),
        ("eps_real_tail", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PSEError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


_lib = None
_VP = ctypes.c_void_p
_SIGS = {
    "pse_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "pse_create": ([ctypes.POINTER(Params), _VP, ctypes.POINTER(_VP)], ctypes.c_int),
    "pse_destroy": ([_VP], ctypes.c_int),
    "pse_get_derived": ([_VP, ctypes.POINTER(Derived)], ctypes.c_int),
    "pse_derive": ([ctypes.POINTER(Params), ctypes.POINTER(Derived)], ctypes.c_int),
    "pse_choose_params": ([ctypes.POINTER(Params), ctypes.POINTER(Tuning), ctypes.POINTER(Params),
                           ctypes.POINTER(TuningInfo)], ctypes.c_int),
    "pse_set_positions": ([_VP, _VP], ctypes.c_int),
    "pse_sample": ([_VP, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, _VP, _VP, ctypes.POINTER(Stats)],
                   ctypes.c_int),
    "pse_sample_with_noise": ([_VP, _VP, _VP, ctypes.c_double, _VP, _VP, ctypes.POINTER(Stats)], ctypes.c_int),
    "pse_bd_step": ([_VP, _VP, _VP, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64, _VP,
                     ctypes.POINTER(Stats)], ctypes.c_int),
    "pse_full_sample": ([_VP, _VP, _VP, ctypes.POINTER(Stats)], ctypes.c_int),
    "pse_real_matvec": ([_VP, _VP, _VP], ctypes.c_int),
    "pse_real_sample": ([_VP, _VP, _VP, ctypes.POINTER(Stats)], ctypes.c_int),
    "pse_wave_sample": ([_VP, _VP, _VP], ctypes.c_int),
    "pse_wave_apply": ([_VP, _VP, _VP], ctypes.c_int),
    "pse_mobility_apply": ([_VP, _VP, _VP], ctypes.c_int),
    "pse_precond_set_weights": ([_VP, _VP, ctypes.c_size_t], ctypes.c_int),
    "pse_precond_set_blocks": ([_VP, _VP], ctypes.c_int),
    "pse_precond_features": ([_VP, _VP], ctypes.c_int),
    "pse_precond_blocks": ([_VP, _VP, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "pse_precond_targets": ([ctypes.POINTER(Params), _VP, _VP, ctypes.c_int32, ctypes.c_double, _VP], ctypes.c_int),
    "pse_mlp_forward": ([_VP, _VP, ctypes.c_int32, _VP, _VP, _VP], ctypes.c_int),
    "pse_mlp_backward_workspace": ([ctypes.c_int32], ctypes.c_size_t),
    "pse_mlp_backward": ([_VP, _VP, _VP, _VP, ctypes.c_int32, _VP, _VP, ctypes.c_size_t, _VP], ctypes.c_int),
    "pse_mlp_backward_noalloc": ([_VP, _VP, _VP, _VP, ctypes.c_int32, _VP, _VP], ctypes.c_int),
    "pse_mlp_adam": ([_VP, _VP, _VP, _VP, _VP, ctypes.c_float, ctypes.c_int32, _VP], ctypes.c_int),
    "pse_mlp_loss_grad": ([_VP, _VP, ctypes.c_int32, _VP, _VP, _VP], ctypes.c_int),
    "pse_batch_create": ([ctypes.POINTER(Params), ctypes.c_int32, _VP, ctypes.POINTER(_VP)], ctypes.c_int),
    "pse_batch_destroy": ([_VP], ctypes.c_int),
    "pse_batch_replica": ([_VP, ctypes.c_int32, ctypes.POINTER(_VP)], ctypes.c_int),
    "pse_batch_set_positions": ([_VP, ctypes.POINTER(_VP)], ctypes.c_int),
    "pse_batch_sample": ([_VP, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(_VP),
                          ctypes.POINTER(_VP), ctypes.POINTER(Stats)], ctypes.c_int),
    "pse_batch_latency": ([_VP, ctypes.POINTER(ctypes.c_float)], ctypes.c_int),
    "pse_batch_graph_create": ([_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.c_double,
                                ctypes.c_int32, ctypes.c_double], ctypes.c_int),
    "pse_batch_graph_step": ([_VP, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(Stats),
                              ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "pse_batch_graph_destroy": ([_VP], ctypes.c_int),
    "pse_batch_autotune": ([_VP], ctypes.c_int),
    "pse_autotune": ([_VP, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "pse_set_launch_shape": ([_VP, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
    "pse_profile": ([_VP, ctypes.c_uint32], ctypes.c_int),
    "pse_profile_read": ([_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
}
STAGES = ("bin", "nbr", "spmv", "lanczos", "noise", "spread", "fft", "xfused", "interp", "other", "precond")
SAMPLE_OK = (PSE_ERR_NOT_CONVERGED, PSE_WARN_PRECOND_FALLBACK)
EXPORTED = tuple(_SIGS)


def load():
    """Load libpse.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} missing (run python paper_1611_09322_amd/build.py)")
        # PyTorch-ROCm ships its own HIP runtime under the same soname; load it
        # first so that the library binds to that one runtime (device pointers
        # and streams from torch are then valid in the library).
        import torch  # noqa: F401

        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def pse_status_string(status):
    return load().pse_status_string(int(status)).decode()


status_string = pse_status_string


def _check(status, where, allow=()):
    if status != PSE_OK and status not in allow:
        raise PSEError(status, where)
    return status


def _ptr(t, dtype, numel, name):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


# --------------------------------------------------------------- C ABI mirror
def pse_create(params, stream=None):
    ctx = _VP()
    _check(load().pse_create(ctypes.byref(params), _VP(stream or 0), ctypes.byref(ctx)), "pse_create")
    return ctx


def pse_destroy(ctx):
    return load().pse_destroy(ctx)


def pse_get_derived(ctx):
    d = Derived()
    _check(load().pse_get_derived(ctx, ctypes.byref(d)), "pse_get_derived")
    return d


def pse_derive(params):
    """Error-model quantities of a parameter set (host only, no GPU)."""
    d = Derived()
    _check(load().pse_derive(ctypes.byref(params), ctypes.byref(d)), "pse_derive")
    return d


def pse_choose_params(base, tuning):
    """(chosen Params, TuningInfo) for a tolerance (host only, no GPU)."""
    out, info = Params(), TuningInfo()
    _check(load().pse_choose_params(ctypes.byref(base), ctypes.byref(tuning), ctypes.byref(out),
                                    ctypes.byref(info)), "pse_choose_params")
    return out, info


def make_params(n, box, a=1.0, eta=1.0, kT=1.0, xi=0.5, rcut=None, grid=64, support=8, gauss_m=0.0, tol=1e-4,
                max_iter=64, precision="fp32", precond=0, flags=0, err_tol=0.0):
    """Params from keyword arguments (rcut defaults to 4 / xi; tol is the
    Lanczos tolerance, err_tol the error-model bound, 0 = unchecked)."""
    if rcut is None:
        rcut = 4.0 / xi
    return Params(int(n), box, a, eta, kT, xi, rcut, int(grid), int(support), gauss_m, tol, int(max_iter),
                  PRECISION[precision] if isinstance(precision, str) else int(precision), int(precond), int(flags),
                  err_tol)


def pse_set_positions(ctx, pos_ptr):
    return _check(load().pse_set_positions(ctx, pos_ptr), "pse_set_positions")


def pse_sample(ctx, seed, counter, dt, forces_ptr, disp_ptr):
    st = Stats()
    s = load().pse_sample(ctx, seed, counter, dt, forces_ptr, disp_ptr, ctypes.byref(st))
    _check(s, "pse_sample", allow=SAMPLE_OK)
    return s, st


def pse_sample_with_noise(ctx, z1_ptr, W_ptr, dt, forces_ptr, disp_ptr):
    st = Stats()
    s = load().pse_sample_with_noise(ctx, z1_ptr, W_ptr, dt, forces_ptr, disp_ptr, ctypes.byref(st))
    _check(s, "pse_sample_with_noise", allow=SAMPLE_OK)
    return s, st


def pse_bd_step(ctx, pos_ptr, forces_ptr, dt, krep, seed, step, disp_ptr):
    st = Stats()
    s = load().pse_bd_step(ctx, pos_ptr, forces_ptr, dt, krep, seed, step, disp_ptr, ctypes.byref(st))
    _check(s, "pse_bd_step", allow=SAMPLE_OK)
    return s, st


def pse_full_sample(ctx, z_ptr, y_ptr):
    st = Stats()
    s = load().pse_full_sample(ctx, z_ptr, y_ptr, ctypes.byref(st))
    _check(s, "pse_full_sample", allow=SAMPLE_OK)
    return s, st


def pse_real_matvec(ctx, v_ptr, w_ptr):
    return _check(load().pse_real_matvec(ctx, v_ptr, w_ptr), "pse_real_matvec")


def pse_real_sample(ctx, z_ptr, y_ptr):
    st = Stats()
    s = load().pse_real_sample(ctx, z_ptr, y_ptr, ctypes.byref(st))
    _check(s, "pse_real_sample", allow=SAMPLE_OK)
    return s, st


def pse_wave_sample(ctx, W_ptr, y_ptr):
    return _check(load().pse_wave_sample(ctx, W_ptr, y_ptr), "pse_wave_sample")


def pse_wave_apply(ctx, f_ptr, u_ptr):
    return _check(load().pse_wave_apply(ctx, f_ptr, u_ptr), "pse_wave_apply")


def pse_mobility_apply(ctx, f_ptr, u_ptr):
    return _check(load().pse_mobility_apply(ctx, f_ptr, u_ptr), "pse_mobility_apply")


def pse_precond_set_weights(ctx, w_bits):
    """w_bits: numpy uint16 array of MLP_NPARAM bf16 bit patterns (host)."""
    import numpy as np

    w = np.ascontiguousarray(w_bits, dtype=np.uint16)
    if w.size != MLP_NPARAM:
        raise ValueError(f"weights must have {MLP_NPARAM} entries")
    return _check(load().pse_precond_set_weights(ctx, w.ctypes.data_as(_VP), w.nbytes), "pse_precond_set_weights")


def pse_precond_set_blocks(ctx, P_ptr):
    return _check(load().pse_precond_set_blocks(ctx, P_ptr), "pse_precond_set_blocks")


def pse_precond_features(ctx, feat_ptr):
    return _check(load().pse_precond_features(ctx, feat_ptr), "pse_precond_features")


def pse_precond_blocks(ctx, P_ptr):
    nf = ctypes.c_int32(0)
    _check(load().pse_precond_blocks(ctx, P_ptr, ctypes.byref(nf)), "pse_precond_blocks")
    return nf.value


def pse_precond_targets(params, pos, idx, radius=0.0):
    """Host FP64 training targets: pos (n, 3) float64, idx int array -> (m, 3, 3)."""
    import numpy as np

    pos = np.ascontiguousarray(pos, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    out = np.empty((len(idx), 9), dtype=np.float64)
    _check(load().pse_precond_targets(ctypes.byref(params), pos.ctypes.data_as(_VP), idx.ctypes.data_as(_VP),
                                      len(idx), radius, out.ctypes.data_as(_VP)), "pse_precond_targets")
    return out.reshape(-1, 3, 3)


def pse_mlp_forward(w_ptr, x_ptr, n, y_ptr, cache_ptr=None, stream=None):
    return _check(load().pse_mlp_forward(w_ptr, x_ptr, n, y_ptr, cache_ptr, _VP(stream or 0)), "pse_mlp_forward")


def pse_mlp_backward_workspace(n):
    return load().pse_mlp_backward_workspace(n)


def pse_mlp_backward(w_ptr, x_ptr, cache_ptr, dy_ptr, n, dw_ptr, work_ptr, work_bytes, stream=None):
    return _check(load().pse_mlp_backward(w_ptr, x_ptr, cache_ptr, dy_ptr, n, dw_ptr, work_ptr, work_bytes,
                                          _VP(stream or 0)), "pse_mlp_backward")


def pse_mlp_backward_noalloc(w_ptr, x_ptr, cache_ptr, dy_ptr, n, dw_ptr, stream=None):
    return _check(load().pse_mlp_backward_noalloc(w_ptr, x_ptr, cache_ptr, dy_ptr, n, dw_ptr, _VP(stream or 0)),
                  "pse_mlp_backward_noalloc")


def pse_mlp_loss_grad(y_ptr, t_ptr, n, dy_ptr, loss_ptr=None, stream=None):
    return _check(load().pse_mlp_loss_grad(y_ptr, t_ptr, n, dy_ptr, loss_ptr, _VP(stream or 0)),
                  "pse_mlp_loss_grad")


def pse_mlp_adam(wm_ptr, wb_ptr, dw_ptr, m_ptr, v_ptr, lr, t, stream=None):
    return _check(load().pse_mlp_adam(wm_ptr, wb_ptr, dw_ptr, m_ptr, v_ptr, lr, t, _VP(stream or 0)),
                  "pse_mlp_adam")


def pse_batch_create(params_list, stream=None):
    arr = (Params * len(params_list))(*params_list)
    b = _VP()
    _check(load().pse_batch_create(arr, len(params_list), _VP(stream or 0), ctypes.byref(b)), "pse_batch_create")
    return b


def pse_batch_destroy(b):
    return load().pse_batch_destroy(b)


def pse_batch_replica(b, r):
    c = _VP()
    _check(load().pse_batch_replica(b, r, ctypes.byref(c)), "pse_batch_replica")
    return c


def pse_batch_set_positions(b, pos_ptrs):
    arr = (_VP * len(pos_ptrs))(*pos_ptrs)
    return _check(load().pse_batch_set_positions(b, arr), "pse_batch_set_positions")


def pse_batch_sample(b, seed, counter, dt, force_ptrs, disp_ptrs):
    n = len(disp_ptrs)
    farr = None if force_ptrs is None else (_VP * n)(*force_ptrs)
    darr = (_VP * n)(*disp_ptrs)
    st = (Stats * n)()
    s = load().pse_batch_sample(b, seed, counter, dt, farr, darr, st)
    _check(s, "pse_batch_sample", allow=SAMPLE_OK)
    return s, list(st)


def pse_batch_graph_create(b, pos_ptrs, force_ptrs, disp_ptrs, dt, extra_iters=4, headroom=0.25):
    n = len(disp_ptrs)
    parr = (_VP * n)(*pos_ptrs)
    farr = None if force_ptrs is None else (_VP * n)(*force_ptrs)
    darr = (_VP * n)(*disp_ptrs)
    _check(load().pse_batch_graph_create(b, parr, farr, darr, dt, extra_iters, headroom), "pse_batch_graph_create")


def pse_batch_graph_step(b, n, seed, counter):
    """One replay; returns (status, per-replica Stats, replicas redone)."""
    st = (Stats * n)()
    red = ctypes.c_int32(0)
    s = load().pse_batch_graph_step(b, seed, counter, st, ctypes.byref(red))
    _check(s, "pse_batch_graph_step", allow=SAMPLE_OK)
    return s, list(st), int(red.value)


def pse_batch_graph_destroy(b):
    _check(load().pse_batch_graph_destroy(b), "pse_batch_graph_destroy")


def pse_batch_latency(b, n):
    ms = (ctypes.c_float * n)()
    _check(load().pse_batch_latency(b, ms), "pse_batch_latency")
    return list(ms)


def pse_autotune(ctx):
    """Pick the fastest spreading tile depth, interpolation workgroup size
    and near-field lanes per target on the current positions; returns
    (depth, interpolation lanes, product lanes per target)."""
    ch = (ctypes.c_int32 * 3)()
    _check(load().pse_autotune(ctx, ch), "pse_autotune")
    return int(ch[0]), int(ch[1]), int(ch[2])


def pse_set_launch_shape(ctx, depth, interp_lanes, product_lanes):
    """Apply a launch-shape choice (0 = built-in for an entry)."""
    ch = (ctypes.c_int32 * 3)(int(depth), int(interp_lanes), int(product_lanes))
    return _check(load().pse_set_launch_shape(ctx, ch), "pse_set_launch_shape")


def pse_batch_autotune(b):
    return _check(load().pse_batch_autotune(b), "pse_batch_autotune")


def pse_profile(ctx, mask):
    return _check(load().pse_profile(ctx, mask), "pse_profile")


def pse_profile_read(ctx):
    ms = (ctypes.c_double * len(STAGES))()
    cnt = (ctypes.c_int32 * len(STAGES))()
    _check(load().pse_profile_read(ctx, ms, cnt), "pse_profile_read")
    return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}


# ----------------------------------------------------------------- wrapper
class Sampler:
    """One sampling context.  Tensors are (n, 3) on the current HIP device;
    the context runs on torch's current stream at construction."""

    def __init__(self, n, box, a=1.0, eta=1.0, kT=1.0, xi=0.5, rcut=None, grid=64, support=8, gauss_m=0.0,
                 tol=1e-4, max_iter=64, precision="fp32", precond=0, stream=None, flags=0, err_tol=0.0,
                 params=None):
        import torch

        self.torch = torch
        if params is None:
            params = make_params(n, box, a, eta, kT, xi, rcut, grid, support, gauss_m, tol, max_iter, precision,
                                 precond, flags, err_tol)
        self.params = params
        self.n = int(params.n)
        self.grid = int(params.grid)
        self.precision = {v: k for k, v in PRECISION.items()}[int(params.precision)]
        self.dtype = torch.float64 if self.precision == "fp64" else torch.float32
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        self.ctx = pse_create(self.params, stream)

    def close(self):
        if getattr(self, "ctx", None):
            pse_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self):
        """Launch-shape autotuning on the current positions: returns the
        spreading tile depth (0 without tiles), the interpolation lanes and
        the near-field product's lanes per target (0 without the LDS path)."""
        return pse_autotune(self.ctx)

    def set_launch_shape(self, depth=0, interp_lanes=0, product_lanes=0):
        """Apply a launch-shape choice without timing (0 = built-in)."""
        pse_set_launch_shape(self.ctx, depth, interp_lanes, product_lanes)

    def profile(self, stages):
        """Time the named stages with HIP events (see STAGES); [] = off."""
        pse_profile(self.ctx, sum(1 << STAGES.index(s) for s in stages))

    def profile_read(self):
        return pse_profile_read(self.ctx)

    def derived(self):
        return pse_get_derived(self.ctx).as_dict()

    def _vec(self, t, name):
        return _ptr(t, self.dtype, 3 * self.n, name)

    def _new(self):
        return self.torch.empty((self.n, 3), dtype=self.dtype, device="cuda")

    def set_positions(self, pos):
        pse_set_positions(self.ctx, self._vec(pos, "positions"))

    def sample(self, seed, counter, dt=1.0, forces=None, out=None):
        out = self._new() if out is None else out
        s, st = pse_sample(self.ctx, seed, counter, dt, self._vec(forces, "forces"), self._vec(out, "out"))
        return out, st

    def _noise(self, W, name="W"):
        """Grid noise W (3, M, M, M) real, or with PSE_FLAG_NOISE_KSPACE zeta
        on the half spectrum (3, M, M, M/2) complex."""
        if W is None:
            return None
        if self.params.flags & FLAG_NOISE_KSPACE:
            ct = self.torch.complex128 if self.dtype == self.torch.float64 else self.torch.complex64
            return _ptr(W, ct, 3 * self.grid * self.grid * (self.grid // 2), name)
        return _ptr(W, self.dtype, 3 * self.grid**3, name)

    def sample_with_noise(self, z1=None, W=None, dt=1.0, forces=None, out=None):
        out = self._new() if out is None else out
        Wp = self._noise(W)
        s, st = pse_sample_with_noise(self.ctx, self._vec(z1, "z1"), Wp, dt, self._vec(forces, "forces"),
                                      self._vec(out, "out"))
        return out, st

    def bd_step(self, pos, seed, step, dt, krep=0.0, forces=None, disp=None):
        """One Euler-Maruyama step in place on pos (n, 3); returns stats."""
        s, st = pse_bd_step(self.ctx, self._vec(pos, "positions"), self._vec(forces, "forces"), dt, krep, seed,
                            step, self._vec(disp, "disp"))
        return st

    def full_sample(self, z, out=None):
        """M^{1/2} z by Lanczos on the whole mobility (flags FLAG_FULL_LANCZOS)."""
        out = self._new() if out is None else out
        s, st = pse_full_sample(self.ctx, self._vec(z, "z"), self._vec(out, "out"))
        return out, st

    def real_matvec(self, v, out=None):
        out = self._new() if out is None else out
        pse_real_matvec(self.ctx, self._vec(v, "v"), self._vec(out, "out"))
        return out

    def real_sample(self, z, out=None):
        out = self._new() if out is None else out
        s, st = pse_real_sample(self.ctx, self._vec(z, "z"), self._vec(out, "out"))
        return out, st

    def wave_sample(self, W, out=None):
        out = self._new() if out is None else out
        pse_wave_sample(self.ctx, self._noise(W), self._vec(out, "out"))
        return out

    def wave_apply(self, F, out=None):
        out = self._new() if out is None else out
        pse_wave_apply(self.ctx, self._vec(F, "forces"), self._vec(out, "out"))
        return out

    def mobility_apply(self, F, out=None):
        out = self._new() if out is None else out
        pse_mobility_apply(self.ctx, self._vec(F, "forces"), self._vec(out, "out"))
        return out

    # learned block preconditioner (precond=1)
    def set_precond_weights(self, w_bits):
        pse_precond_set_weights(self.ctx, w_bits)

    def set_precond_blocks(self, P):
        """Use the (n, 3, 3) float32 blocks P (caller order) in place of the
        network's until set_precond_weights; None returns to the network."""
        pse_precond_set_blocks(self.ctx, None if P is None else _ptr(P, self.torch.float32, 9 * self.n, "P"))

    def precond_features(self, out=None):
        """(n, 24) bfloat16 features of the current positions (caller order)."""
        out = self.torch.empty((self.n, 24), dtype=self.torch.bfloat16, device="cuda") if out is None else out
        pse_precond_features(self.ctx, _ptr(out, self.torch.bfloat16, 24 * self.n, "out"))
        return out

    def precond_blocks(self, out=None):
        """((n, 3, 3) float32 blocks in use, number of fallback blocks)."""
        out = self.torch.empty((self.n, 3, 3), dtype=self.torch.float32, device="cuda") if out is None else out
        nf = pse_precond_blocks(self.ctx, _ptr(out, self.torch.float32, 9 * self.n, "out"))
        return out, nf


class Batch:
    """Independent replicas sampled together (pse_batch_*).  `specs` is a
    list of dicts with the Sampler keyword arguments plus n and box."""

    def __init__(self, specs, stream=None):
        import torch

        self.torch = torch
        self.params = []
        self.n = []
        self.dtypes = []
        for sp in specs:
            prec = sp.get("precision", "fp32")
            rc = sp.get("rcut") or 4.0 / sp.get("xi", 0.5)
            self.params.append(Params(int(sp["n"]), sp["box"], sp.get("a", 1.0), sp.get("eta", 1.0),
                                      sp.get("kT", 1.0), sp.get("xi", 0.5), rc, int(sp.get("grid", 64)),
                                      int(sp.get("support", 8)), sp.get("gauss_m", 0.0), sp.get("tol", 1e-4),
                                      int(sp.get("max_iter", 64)), PRECISION[prec], int(sp.get("precond", 0)),
                                      int(sp.get("flags", 0)), sp.get("err_tol", 0.0)))
            self.n.append(int(sp["n"]))
            self.dtypes.append(torch.float64 if prec == "fp64" else torch.float32)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.b = pse_batch_create(self.params, stream)

    def close(self):
        if getattr(self, "b", None):
            pse_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _ptrs(self, ts, name):
        return [_ptr(t, dt, 3 * n, f"{name}[{r}]") for r, (t, dt, n) in enumerate(zip(ts, self.dtypes, self.n))]

    def set_positions(self, pos):
        pse_batch_set_positions(self.b, self._ptrs(pos, "positions"))

    def sample(self, seed, counter, dt=1.0, forces=None, out=None):
        if out is None:
            out = [self.torch.empty((n, 3), dtype=dt_, device="cuda") for n, dt_ in zip(self.n, self.dtypes)]
        fp = None if forces is None else self._ptrs(forces, "forces")
        s, st = pse_batch_sample(self.b, seed, counter, dt, fp, self._ptrs(out, "out"))
        return out, st

    def latency(self):
        return pse_batch_latency(self.b, len(self.n))

    def graph_create(self, pos, out, dt, forces=None, extra_iters=4, headroom=0.25):
        """Capture one step (set positions + sample) on these buffers
        (pse_batch_graph_create); the tensors must outlive the graph."""
        fp = None if forces is None else self._ptrs(forces, "forces")
        self._graph_bufs = (pos, out, forces)
        pse_batch_graph_create(self.b, self._ptrs(pos, "positions"), fp, self._ptrs(out, "out"), dt, extra_iters,
                               headroom)

    def graph_step(self, seed, counter):
        """One replay: (status, stats, replicas redone)."""
        return pse_batch_graph_step(self.b, len(self.n), seed, counter)

    def graph_destroy(self):
        pse_batch_graph_destroy(self.b)
        self._graph_bufs = None

    def autotune(self):
        """pse_batch_autotune (after set_positions)."""
        pse_batch_autotune(self.b)

    def set_precond_weights(self, r, w_bits):
        """Learned-preconditioner weights of replica r (created with precond=1)."""
        pse_precond_set_weights(pse_batch_replica(self.b, r), w_bits)
