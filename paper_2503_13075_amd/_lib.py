"""ctypes binding of ``libilves.so`` (argument marshalling only).

Every step of the solve runs in the library's HIP kernels; PyTorch only
provides device memory (tensors passed by ``data_ptr()``) and streams.
Nothing here falls back to a CPU implementation: if the library is missing
the import of the solver fails loudly.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libilves.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "ilves.h")

OK, ERR_ARG, ERR_TOPOLOGY, ERR_HIP, ERR_NOMEM, ERR_SINGULAR, ERR_NOT_CONVERGED, ERR_NONFINITE, ERR_UNSUPPORTED, ERR_TIMEOUT = range(10)
PREC_FP64, PREC_MIXED = 0, 1
VARIANT_NEWTON, VARIANT_CHORD = 0, 1
WARM_ZERO, WARM_MLP, WARM_CALLER, WARM_DECOUPLED = 0, 1, 2, 3
STAT_NAMES = ["molecules", "constraints", "atoms", "factor_entries", "fill", "updates", "max_levels",
              "sum_levels", "mol_lds", "mol_workspace", "workspace_bytes", "plan_bytes", "split_molecules",
              "split_parts", "max_separator", "split_values_lds", "split_pairs_global",
              "split_shared_lane_levels"]


class IlvesError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ilves error {code}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("variant", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("block_threads", ctypes.c_int32), ("lds_limit", ctypes.c_int32),
                ("ordering", ctypes.c_int32), ("split_rows", ctypes.c_int32), ("split_part_rows", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("band_block", ctypes.c_int32 * 5), ("lds_limit", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


_lib = None
_P = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_I64P = ctypes.POINTER(ctypes.c_int64)
_F64P = ctypes.POINTER(ctypes.c_double)
_F32P = ctypes.POINTER(ctypes.c_float)


def header_functions() -> list:
    """Names of the functions that include/ilves.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ilves_[a-z_]+)\s*\(", txt)))


def lib() -> ctypes.CDLL:
    """Loads the library once.  torch is imported first so that the process
    has a single HIP runtime (the library's libamdhip64.so.7 dependency then
    resolves to the copy torch already loaded)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (HIP runtime first)
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2503_13075_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.ilves_default_options.argtypes = [ctypes.POINTER(Options)]
    L.ilves_default_options.restype = None
    L.ilves_version.restype = ctypes.c_char_p
    L.ilves_last_error.restype = ctypes.c_char_p
    L.ilves_status_string.argtypes = [ctypes.c_int]
    L.ilves_status_string.restype = ctypes.c_char_p
    L.ilves_plan_create.argtypes = [ctypes.c_int32, ctypes.c_int32, _I32P, _F64P, ctypes.POINTER(Options),
                                    ctypes.POINTER(_P)]
    L.ilves_plan_create.restype = ctypes.c_int
    L.ilves_plan_destroy.argtypes = [_P]
    L.ilves_plan_destroy.restype = ctypes.c_int
    L.ilves_plan_num_molecules.argtypes = [_P]
    L.ilves_plan_num_molecules.restype = ctypes.c_int32
    L.ilves_project_velocities.argtypes = [_P, _P, _P, _P, ctypes.c_double, ctypes.c_int32, _P, _P, _P, _P, _P]
    L.ilves_project_velocities.restype = ctypes.c_int
    L.ilves_plan_set_wait_limit.argtypes = [_P, ctypes.c_int32]
    L.ilves_plan_set_wait_limit.restype = ctypes.c_int
    L.ilves_plan_reset_barriers.argtypes = [_P]
    L.ilves_plan_reset_barriers.restype = ctypes.c_int
    L.ilves_plan_stats.argtypes = [_P, _I64P]
    L.ilves_plan_stats.restype = ctypes.c_int
    L.ilves_plan_molecules.argtypes = [_P, _I32P, _I32P, _I32P, _I32P]
    L.ilves_plan_molecules.restype = ctypes.c_int
    L.ilves_solve.argtypes = [_P, _P, _P, _P, ctypes.c_double, _P, _P, _P, _P, _P]
    L.ilves_solve.restype = ctypes.c_int
    L.ilves_solve_ex.argtypes = [_P, _P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, _P, _P, _P, _P, _P, ctypes.c_int32, _P]
    L.ilves_solve_ex.restype = ctypes.c_int
    L.ilves_plan_replay_host.argtypes = [ctypes.c_int32, ctypes.c_int32, _I32P, _F64P, ctypes.POINTER(Options),
                                         _F64P, _F64P, _F64P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, _F64P, _F64P, _I32P, _I32P, _I32P, _I64P]
    L.ilves_plan_replay_host.restype = ctypes.c_int
    L.ilves_mlp_param_count.restype = ctypes.c_int32
    L.ilves_mlp_norm_count.restype = ctypes.c_int32
    L.ilves_mlp_load.argtypes = [_P, _F32P, ctypes.c_int32, _F32P, ctypes.c_int32]
    L.ilves_mlp_load.restype = ctypes.c_int
    L.ilves_features.argtypes = [_P, _P, _P, _P, _P, _P, _P]
    L.ilves_features.restype = ctypes.c_int
    L.ilves_plan_row_constraints.argtypes = [_P, _I32P]
    L.ilves_plan_row_constraints.restype = ctypes.c_int
    L.ilves_mlp_predict.argtypes = [_P, _P, _P, _P, _P, _P]
    L.ilves_mlp_predict.restype = ctypes.c_int
    L.ilves_solve_learned.argtypes = [_P, _P, _P, _P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, _P, _P, _P, _P, _P, _P]
    L.ilves_solve_learned.restype = ctypes.c_int
    L.ilves_mlp_forward_f32.argtypes = [_P, _P, ctypes.c_int32, _P, _P]
    L.ilves_mlp_forward_f32.restype = ctypes.c_int
    L.ilves_mlp_grad_workspace.argtypes = [ctypes.c_int32]
    L.ilves_mlp_grad_workspace.restype = ctypes.c_int64
    L.ilves_mlp_grad_f32.argtypes = [_P, _P, _P, ctypes.c_int32, _P, _P, _P, ctypes.c_int64, _P]
    L.ilves_mlp_grad_f32.restype = ctypes.c_int
    L.ilves_mlp_grad_f32_static.argtypes = [_P, _P, _P, ctypes.c_int32, _P, _P, _P]
    L.ilves_mlp_grad_f32_static.restype = ctypes.c_int
    L.ilves_mlp_adam_f32.argtypes = [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_int32, _P]
    L.ilves_mlp_adam_f32.restype = ctypes.c_int
    L.ilves_perturb_normal.argtypes = [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, _P, _P, _P]
    L.ilves_perturb_normal.restype = ctypes.c_int
    L.ilves_counter_add.argtypes = [_P, ctypes.c_uint64, _P]
    L.ilves_md_kick_drift.argtypes = [_P, _P, _P, _P, ctypes.c_double, ctypes.c_int32, _P, _P]
    L.ilves_md_kick_drift.restype = ctypes.c_int
    L.ilves_md_finish.argtypes = [_P, _P, ctypes.c_double, ctypes.c_int32, _P, _P]
    L.ilves_md_finish.restype = ctypes.c_int
    L.ilves_counter_add.restype = ctypes.c_int
    L.ilves_plan_get_tuning.argtypes = [_P, ctypes.POINTER(Tuning)]
    L.ilves_plan_get_tuning.restype = ctypes.c_int
    L.ilves_plan_tune.argtypes = [_P, ctypes.POINTER(Tuning)]
    L.ilves_plan_tune.restype = ctypes.c_int
    _lib = L
    return L


def check(code: int):
    if code != OK:
        raise IlvesError(code, lib().ilves_last_error().decode())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def make_options(precision=PREC_FP64, variant=VARIANT_NEWTON, max_iter=0, warm_start=WARM_ZERO,
                 block_threads=0, lds_limit=0, ordering=0, split_rows=0, split_part_rows=0) -> Options:
    o = Options()
    lib().ilves_default_options(ctypes.byref(o))
    o.precision, o.variant, o.max_iter, o.warm_start = precision, variant, max_iter, warm_start
    o.block_threads, o.lds_limit, o.ordering = block_threads, lds_limit, ordering
    o.split_rows, o.split_part_rows = split_rows, split_part_rows
    return o


def _topology(pairs, d):
    pairs = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(-1))
    if pairs.shape[0] != d.shape[0]:
        raise ValueError("pairs and d have different lengths")
    return pairs, d


def replay_host(n_atoms, pairs, d, mass, r_soa, ru_soa, tol, precision=PREC_FP64, variant=VARIANT_NEWTON,
                max_iter=0, ordering=0, split_rows=0, split_part_rows=0):
    """Runs the planner and replays the device schedule on the host
    (planner diagnostics; see ilves_plan_replay_host)."""
    L = lib()
    pairs, d = _topology(pairs, d)
    n = pairs.shape[0]
    mass = np.ascontiguousarray(mass, dtype=np.float64)
    r_soa = np.ascontiguousarray(r_soa, dtype=np.float64)
    ru_soa = np.ascontiguousarray(ru_soa, dtype=np.float64)
    r_out = np.zeros_like(ru_soa)
    lam = np.zeros(n)
    iters = np.zeros(max(n, 1), np.int32)
    status = np.zeros(max(n, 1), np.int32)
    nm = ctypes.c_int32(0)
    st = np.zeros(6, np.int64)
    o = make_options(ordering=ordering, split_rows=split_rows, split_part_rows=split_part_rows)
    check(L.ilves_plan_replay_host(n_atoms, n, _ptr(pairs, ctypes.c_int32), _ptr(d, ctypes.c_double), ctypes.byref(o),
                                   _ptr(mass, ctypes.c_double), _ptr(r_soa, ctypes.c_double),
                                   _ptr(ru_soa, ctypes.c_double), tol, precision, variant, max_iter,
                                   _ptr(r_out, ctypes.c_double), _ptr(lam, ctypes.c_double),
                                   _ptr(iters, ctypes.c_int32), _ptr(status, ctypes.c_int32), ctypes.byref(nm),
                                   _ptr(st, ctypes.c_int64)))
    k = nm.value
    return {"r_out": r_out, "lam": lam, "iters": iters[:k].copy(), "status": status[:k].copy(),
            "stats": dict(zip(["molecules", "factor_entries", "updates", "max_levels", "fill", "split"], st.tolist()))}


class Plan:
    """A planned topology on the current GPU (wraps ilves_plan_create)."""

    def __init__(self, n_atoms, pairs, d, precision=PREC_FP64, variant=VARIANT_NEWTON, max_iter=0,
                 warm_start=WARM_ZERO, block_threads=0, lds_limit=0, ordering=0, split_rows=0, split_part_rows=0):
        L = lib()
        self._L = L
        pairs, d = _topology(pairs, d)
        self.n_atoms = int(n_atoms)
        self.n_constraints = int(pairs.shape[0])
        o = make_options(precision, variant, max_iter, warm_start, block_threads, lds_limit, ordering, split_rows,
                         split_part_rows)
        h = _P()
        check(L.ilves_plan_create(self.n_atoms, self.n_constraints, _ptr(pairs, ctypes.c_int32),
                                  _ptr(d, ctypes.c_double), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self.n_molecules = int(L.ilves_plan_num_molecules(h))

    def close(self):
        if getattr(self, "_h", None):
            self._L.ilves_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def project_velocities(self, r, v, mass, tol, v_out, mu, iters, status, precision=PREC_FP64, stream=None):
        """Velocity constraints (RATTLE's velocity half): v_out = v - M^-1
        G(r)^T mu with G(r) v_out = 0.  Device tensors as for solve (v, v_out
        float64 [3, n_atoms], mu float64 [n_constraints])."""
        import torch
        for t, dt in ((r, torch.float64), (v, torch.float64), (mass, torch.float64), (v_out, torch.float64),
                      (mu, torch.float64), (iters, torch.int32), (status, torch.int32)):
            if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
                raise ValueError("project_velocities expects contiguous device tensors of the documented dtypes")
        if r.shape != (3, self.n_atoms) or v.shape != (3, self.n_atoms) or v_out.shape != (3, self.n_atoms):
            raise ValueError("positions and velocities must have shape [3, n_atoms]")
        if mass.shape != (self.n_atoms,) or mu.shape != (self.n_constraints,):
            raise ValueError("mass / mu have the wrong length")
        if iters.numel() < self.n_molecules or status.numel() < self.n_molecules:
            raise ValueError("iters / status need one entry per molecule")
        if stream is None:
            stream = torch.cuda.current_stream()
        check(self._L.ilves_project_velocities(self._h, r.data_ptr(), v.data_ptr(), mass.data_ptr(), float(tol),
                                               precision, v_out.data_ptr(), mu.data_ptr(), iters.data_ptr(),
                                               status.data_ptr(), ctypes.c_void_p(stream.cuda_stream)))

    def set_wait_limit(self, polls: int):
        """Bound on the polls of a split molecule's barrier wait (see
        ilves_plan_set_wait_limit)."""
        check(self._L.ilves_plan_set_wait_limit(self._h, int(polls)))

    def reset_barriers(self):
        """Clears the barrier state of every split molecule (after
        ILVES_ERR_TIMEOUT); synchronises the device (see
        ilves_plan_reset_barriers)."""
        check(self._L.ilves_plan_reset_barriers(self._h))

    def stats(self) -> dict:
        st = np.zeros(len(STAT_NAMES), np.int64)
        check(self._L.ilves_plan_stats(self._h, _ptr(st, ctypes.c_int64)))
        return dict(zip(STAT_NAMES, st.tolist()))

    def molecules(self) -> dict:
        k = self.n_molecules
        a = [np.zeros(max(k, 1), np.int32) for _ in range(4)]
        check(self._L.ilves_plan_molecules(self._h, *[_ptr(x, ctypes.c_int32) for x in a]))
        return {"n_con": a[0][:k], "n_atoms": a[1][:k], "n_levels": a[2][:k], "first_constraint": a[3][:k]}

    def solve(self, r, r_u, mass, tol, r_out, lam, iters, status, precision=PREC_FP64, variant=VARIANT_NEWTON,
              warm_start=WARM_ZERO, max_iter=0, stream=None, history=None):
        """Enqueues one solve.  All tensors are CUDA (HIP) tensors: r, r_u,
        r_out float64 [3, n_atoms] contiguous, mass float64 [n_atoms], lam
        float64 [n_constraints], iters/status int32 [n_molecules]; history
        (optional) float64 [n_molecules, L] receives each molecule's maximum
        relative violation at iterates 0 .. L-1."""
        import torch
        for t, dt in ((r, torch.float64), (r_u, torch.float64), (mass, torch.float64), (r_out, torch.float64),
                      (lam, torch.float64), (iters, torch.int32), (status, torch.int32)):
            if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
                raise ValueError("solve expects contiguous device tensors of the documented dtypes")
        if r.shape != (3, self.n_atoms) or r_u.shape != (3, self.n_atoms) or r_out.shape != (3, self.n_atoms):
            raise ValueError("positions must have shape [3, n_atoms]")
        if mass.shape != (self.n_atoms,) or lam.shape != (self.n_constraints,):
            raise ValueError("mass / lambda have the wrong length")
        if iters.numel() < self.n_molecules or status.numel() < self.n_molecules:
            raise ValueError("iters / status need one entry per molecule")
        h_ptr, h_len = None, 0
        if history is not None:
            if not history.is_cuda or history.dtype != torch.float64 or not history.is_contiguous() or \
                    history.dim() != 2 or history.shape[0] < self.n_molecules:
                raise ValueError("history must be a contiguous float64 device tensor [n_molecules, L]")
            h_ptr, h_len = history.data_ptr(), int(history.shape[1])
        if stream is None:
            stream = torch.cuda.current_stream()
        check(self._L.ilves_solve_ex(self._h, r.data_ptr(), r_u.data_ptr(), mass.data_ptr(), float(tol), precision,
                                     variant, warm_start, max_iter, r_out.data_ptr(), lam.data_ptr(),
                                     iters.data_ptr(), status.data_ptr(), h_ptr, h_len,
                                     ctypes.c_void_p(stream.cuda_stream)))


def _stream(stream):
    import torch
    return ctypes.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)


def _dev(t, dtype, shape=None):
    import torch
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor of dtype %s" % dtype)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t.data_ptr()


def mlp_param_count() -> int:
    return int(lib().ilves_mlp_param_count())


def mlp_norm_count() -> int:
    return int(lib().ilves_mlp_norm_count())


def mlp_forward_f32(params, x, out, stream=None):
    """FP32 forward pass of normalised inputs x [n, 16] (device tensors)."""
    import torch
    n = x.shape[0]
    check(lib().ilves_mlp_forward_f32(_dev(params, torch.float32), _dev(x, torch.float32, (n, 16)), n,
                                      _dev(out, torch.float32, (n,)), _stream(stream)))


def mlp_grad_f32(params, x, y, grad, loss, work, stream=None):
    """Gradient of 1/(2n) sum (out - y)^2 (device tensors)."""
    import torch
    n = x.shape[0]
    check(lib().ilves_mlp_grad_f32(_dev(params, torch.float32), _dev(x, torch.float32, (n, 16)),
                                   _dev(y, torch.float32, (n,)), n, _dev(grad, torch.float32),
                                   _dev(loss, torch.float32), _dev(work, torch.float32), work.numel(),
                                   _stream(stream)))


# sample limit of ilves_mlp_grad_f32_static, as include/ilves.h defines it
MLP_GRAD_STATIC_MAX_SAMPLES = int(re.search(r"#define ILVES_MLP_GRAD_STATIC_MAX_SAMPLES (\d+)",
                                            open(HEADER).read()).group(1))


def mlp_grad_f32_static(params, x, y, grad, loss, stream=None):
    """The gradient of mlp_grad_f32 without a workspace: the library's fixed
    device array holds the partial sums (at most MLP_GRAD_STATIC_MAX_SAMPLES
    samples; calls that overlap on one GPU race)."""
    import torch
    n = x.shape[0]
    check(lib().ilves_mlp_grad_f32_static(_dev(params, torch.float32), _dev(x, torch.float32, (n, 16)),
                                          _dev(y, torch.float32, (n,)), n, _dev(grad, torch.float32),
                                          _dev(loss, torch.float32), _stream(stream)))


def mlp_grad_workspace(n) -> int:
    return int(lib().ilves_mlp_grad_workspace(int(n)))


def mlp_adam(params, grad, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    import torch
    check(lib().ilves_mlp_adam_f32(_dev(params, torch.float32), _dev(grad, torch.float32), _dev(m, torch.float32),
                                   _dev(v, torch.float32), params.numel(), lr, beta1, beta2, eps, int(step),
                                   _stream(stream)))


def _plan_load_mlp(self, params, norm):
    """Loads network parameters and normalisation (host float arrays)."""
    params = np.ascontiguousarray(params, dtype=np.float32)
    norm = np.ascontiguousarray(norm, dtype=np.float32)
    if params.size != mlp_param_count() or norm.size != mlp_norm_count():
        raise ValueError("wrong parameter or normalisation size")
    check(self._L.ilves_mlp_load(self._h, _ptr(params, ctypes.c_float), params.size, _ptr(norm, ctypes.c_float),
                                 norm.size))


def _plan_row_constraints(self):
    out = np.zeros(max(1, self.n_constraints), np.int32)
    check(self._L.ilves_plan_row_constraints(self._h, _ptr(out, ctypes.c_int32)))
    return out[:self.n_constraints]


def _plan_features(self, r, r_u, mass, feat, w, stream=None):
    import torch
    check(self._L.ilves_features(self._h, _dev(r, torch.float64, (3, self.n_atoms)),
                                 _dev(r_u, torch.float64, (3, self.n_atoms)), _dev(mass, torch.float64),
                                 _dev(feat, torch.float32, (self.n_constraints, 16)),
                                 _dev(w, torch.float32, (self.n_constraints,)), _stream(stream)))


def _plan_predict(self, r, r_u, mass, lam, stream=None):
    import torch
    check(self._L.ilves_mlp_predict(self._h, _dev(r, torch.float64, (3, self.n_atoms)),
                                    _dev(r_u, torch.float64, (3, self.n_atoms)), _dev(mass, torch.float64),
                                    _dev(lam, torch.float64, (self.n_constraints,)), _stream(stream)))


def _plan_solve_learned(self, r, r_u, mass, tol, r_out, lam, iters, status, fallback=None, precision=PREC_MIXED,
                        variant=VARIANT_NEWTON, max_iter=0, stream=None):
    import torch
    fb = 0 if fallback is None else _dev(fallback, torch.int32)
    check(self._L.ilves_solve_learned(self._h, _dev(r, torch.float64, (3, self.n_atoms)),
                                      _dev(r_u, torch.float64, (3, self.n_atoms)), _dev(mass, torch.float64),
                                      float(tol), precision, variant, max_iter,
                                      _dev(r_out, torch.float64, (3, self.n_atoms)),
                                      _dev(lam, torch.float64, (self.n_constraints,)), _dev(iters, torch.int32),
                                      _dev(status, torch.int32), fb, _stream(stream)))


def _plan_get_tuning(self) -> dict:
    t = Tuning()
    check(self._L.ilves_plan_get_tuning(self._h, ctypes.byref(t)))
    return {"band_block": list(t.band_block), "lds_limit": int(t.lds_limit)}


def _plan_tune(self, band_block=None, lds_limit=None):
    """Re-derives placement and launch groups (block size per LDS band, LDS
    limit per molecule).  Synchronises the device; graphs captured before
    must be captured again."""
    cur = self.get_tuning()
    t = Tuning()
    for i, b in enumerate(cur["band_block"] if band_block is None else band_block):
        t.band_block[i] = int(b)
    t.lds_limit = int(cur["lds_limit"] if lds_limit is None else lds_limit)
    check(self._L.ilves_plan_tune(self._h, ctypes.byref(t)))


def perturb_normal(r, sigma, seed, step, r_u, stream=None):
    """r_u = r + sigma * z on the device (Philox4x32-10 + Box-Muller); r and
    r_u float64 [3, n_atoms] CUDA tensors, step a uint64-sized int64 CUDA
    tensor of one element holding the step index."""
    import torch
    n = r.shape[1]
    check(lib().ilves_perturb_normal(_dev(r, torch.float64, (3, n)), n, float(sigma), int(seed) & (2**64 - 1),
                                     _dev(step, torch.int64, (1,)), _dev(r_u, torch.float64, (3, n)),
                                     _stream(stream)))


def md_kick_drift(r, v, f, mass, h, r_u, stream=None):
    """v += h f / m; r_u = r + h v (float64 CUDA tensors, SoA [3, n])."""
    import torch
    n = r.shape[1]
    check(lib().ilves_md_kick_drift(_dev(r, torch.float64, (3, n)), _dev(v, torch.float64, (3, n)),
                                    _dev(f, torch.float64, (3, n)), _dev(mass, torch.float64, (n,)), float(h), n,
                                    _dev(r_u, torch.float64, (3, n)), _stream(stream)))


def md_finish(r, r_new, h, v, stream=None):
    """v = (r_new - r) / h; r = r_new."""
    import torch
    n = r.shape[1]
    check(lib().ilves_md_finish(_dev(r, torch.float64, (3, n)), _dev(r_new, torch.float64, (3, n)), float(h), n,
                                _dev(v, torch.float64, (3, n)), _stream(stream)))


def counter_add(counter, delta=1, stream=None):
    import torch
    check(lib().ilves_counter_add(_dev(counter, torch.int64, (1,)), int(delta), _stream(stream)))


Plan.get_tuning = _plan_get_tuning
Plan.tune = _plan_tune
Plan.load_mlp = _plan_load_mlp
Plan.row_constraints = _plan_row_constraints
Plan.features = _plan_features
Plan.predict = _plan_predict
Plan.solve_learned = _plan_solve_learned
