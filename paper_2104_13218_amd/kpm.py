"""Python binding of the C ABI in include/kpm.h (ctypes; argument marshalling only).

Every computation runs in libkpm.so on the GPU.  PyTorch provides device
memory (tensors whose data pointers are passed through) and the stream
(torch's current stream).  If the library is not built, `load()` raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, c_double, c_int32, c_int64, c_size_t, c_uint8, c_uint32, c_uint64, c_void_p

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# KPM_LIBRARY names another build of the same library (the sanitized one)
LIB_PATH = os.environ.get("KPM_LIBRARY") or os.path.join(_HERE, "libkpm.so")

KPM_OK, KPM_EINVAL, KPM_ENOMEM, KPM_EDEVICE, KPM_EBOUNDS, KPM_EWORKSPACE = 0, -1, -2, -3, -4, -5
KPM_ETOOLARGE = -6
NOALLOC_MAX_BYTES = 64 << 20  # KPM_NOALLOC_MAX_BYTES of include/kpm.h
VEC_KINDS = {"rademacher": 0, "complex_gaussian": 1, "gaussian": 2, "basis": 3}
PRECISIONS = {"fp64": 0, "fp32": 1, "fp32r": 2}   # fp32r: float32 + 16-bit residual storage
KERNELS = {"none": 0, "jackson": 1}


class KPMError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class Problem(ctypes.Structure):
    _fields_ = [("n_sites", c_int32), ("n_up", c_int32), ("n_bonds", c_int32), ("cluster", c_int32),
                ("bond_i", POINTER(c_int32)), ("bond_j", POINTER(c_int32)), ("J", POINTER(c_double)),
                ("e_lo", c_double), ("e_hi", c_double), ("two_s", c_int32), ("reserved", c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("eps", c_double), ("M", c_int32), ("R", c_int32), ("vec_kind", c_int32),
                ("precision", c_int32), ("col_block", c_int32), ("seed", c_uint64),
                ("lanczos_steps", c_int32), ("bound_margin", c_double), ("autotune", c_int32)]


class RunStats(ctypes.Structure):
    _fields_ = [("step_launches", c_int64), ("bytes_per_launch", c_double),
                ("state_col_steps", c_double), ("col_block", c_int32), ("rows_per_tile", c_int32),
                ("graph_segment", c_int32), ("kernel", c_int32), ("recursion_ms", c_double),
                ("relabelled", c_int32), ("waves", c_int32)]


_lib = None

_SIGS = {
    "kpm_strerror": (ctypes.c_char_p, [c_int32]),
    "kpm_sector_dim": (c_uint64, [c_int32, c_int32]),
    "kpm_sector_states": (c_int32, [c_int32, c_int32, c_void_p, c_void_p]),
    "kpm_sector_matrix": (c_int32, [POINTER(Problem), c_int64, c_int64, c_int32, c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_void_p]),
    "kpm_spectral_bounds": (c_int32, [POINTER(Problem), c_int32, c_int32, c_double, c_uint64,
                                      POINTER(c_double), c_void_p]),
    "chebyshev_moments_workspace_size": (c_size_t, [POINTER(Problem), c_int32, POINTER(Params)]),
    "chebyshev_moments": (c_int32, [POINTER(Problem), c_int32, POINTER(Params), c_void_p, c_void_p,
                                    c_void_p, c_size_t, c_void_p]),
    "chebyshev_moments_noalloc": (c_int32, [POINTER(Problem), c_int32, POINTER(Params), c_void_p,
                                            c_void_p, c_void_p]),
    "chebyshev_vectors_workspace_size": (c_size_t, [POINTER(Problem), POINTER(Params), c_int32]),
    "chebyshev_vectors": (c_int32, [POINTER(Problem), POINTER(Params), c_int32, c_void_p, c_void_p,
                                    c_void_p, c_size_t, c_void_p]),
    "kpm_thermo": (c_int32, [c_void_p, c_void_p, POINTER(Problem), c_int32, c_int32, c_int32, c_int32,
                             c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                             c_void_p]),
    "kpm_thermo_field": (c_int32, [c_void_p, c_void_p, POINTER(Problem), c_int32, c_int32, c_int32,
                                   c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_void_p]),
    "kpm_ftlm_workspace_size": (c_size_t, [POINTER(Problem), c_int32, POINTER(Params)]),
    "kpm_ftlm": (c_int32, [POINTER(Problem), c_int32, POINTER(Params), c_void_p, c_void_p, c_int32,
                           c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                           c_void_p, c_size_t, c_void_p]),
    "kpm_sector_eigenvalues_workspace_size": (c_size_t, [POINTER(Problem), c_int32, c_int32]),
    "kpm_sector_eigenvalues": (c_int32, [POINTER(Problem), c_int32, c_int32, c_void_p, c_void_p, c_size_t,
                                         c_void_p]),
    "kpm_thermo_hybrid": (c_int32, [c_void_p, c_void_p, POINTER(Problem), c_int32, c_int32, c_int32, c_int32,
                                    c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                    c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "kpm_thermo_vjp": (c_int32, [c_void_p, c_void_p, POINTER(Problem), c_int32, c_int32, c_int32,
                                 c_int32, c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "chebyshev_moments_vjp_workspace_size": (c_size_t, [POINTER(Problem), c_int32, POINTER(Params),
                                                        c_int32]),
    "chebyshev_moments_vjp": (c_int32, [POINTER(Problem), c_int32, POINTER(Params), c_void_p, c_void_p,
                                        c_int32, c_void_p, c_void_p, c_size_t, c_void_p]),
    "chebyshev_moments_ckpt_workspace_size": (c_size_t, [POINTER(Problem), c_int32, POINTER(Params),
                                                         c_int32]),
    "chebyshev_moments_ckpt": (c_int32, [POINTER(Problem), c_int32, POINTER(Params), c_int32, c_void_p,
                                         c_void_p, c_void_p, c_size_t, c_void_p]),
    "chebyshev_moments_vjp_resume": (c_int32, [POINTER(Problem), c_int32, POINTER(Params), c_void_p,
                                               c_void_p, c_int32, c_void_p, c_void_p, c_size_t, c_void_p]),
    "kpm_thermo_grad": (c_int32, [POINTER(Problem), c_int32, POINTER(Params), c_int32, c_int32,
                                  c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_size_t, c_void_p]),
    "kpm_cluster_bond_grad": (c_int32, [POINTER(Problem), c_int32, c_void_p, c_void_p, c_void_p]),
    "kpm_last_run_stats": (c_int32, [POINTER(RunStats)]),
    "kpm_site_relabel": (c_int32, [POINTER(Problem), c_int32, POINTER(c_int32)]),
    "kpm_autotune_reset": (c_int32, []),
}


def load():
    """Load libkpm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2104_13218_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def strerror(code: int) -> str:
    return load().kpm_strerror(code).decode()


def _f64(x):
    """x as a contiguous float64 CUDA tensor (the ABI's double arrays)."""
    return torch.as_tensor(x, dtype=torch.float64, device="cuda").contiguous()


def _check(code: int, what: str):
    if code != KPM_OK:
        raise KPMError(code, what)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


class ProblemSet:
    """ctypes array of kpm_problem built from workloads.Sector objects (keeps
    the bond arrays alive)."""

    def __init__(self, sectors, bounds=None):
        self.sectors = list(sectors)
        n = len(self.sectors)
        self.arr = (Problem * n)()
        self._keep = []
        for k, s in enumerate(self.sectors):
            c = s.cluster
            bi = np.ascontiguousarray(c.bond_i, dtype=np.int32)
            bj = np.ascontiguousarray(c.bond_j, dtype=np.int32)
            J = np.ascontiguousarray(c.J, dtype=np.float64)
            self._keep += [bi, bj, J]
            if bounds is not None and bounds[k] is not None:
                lo, hi = bounds[k]
            else:
                lo, hi = float(getattr(s, "e_lo", float("nan"))), float(getattr(s, "e_hi", float("nan")))
            self.arr[k] = Problem(c.n_sites, s.n_up, c.n_bonds, s.cluster_id,
                                  bi.ctypes.data_as(POINTER(c_int32)), bj.ctypes.data_as(POINTER(c_int32)),
                                  J.ctypes.data_as(POINTER(c_double)), lo, hi, int(getattr(s, "two_s", 1)), 0)

    def __len__(self):
        return len(self.sectors)

    @property
    def n_clusters(self):
        return 1 + max(s.cluster_id for s in self.sectors)


def make_params(M, R=1, vec_kind="rademacher", precision="fp64", eps=0.025, seed=0, col_block=0,
                lanczos_steps=50, margin=0.01, autotune=False) -> Params:
    return Params(float(eps), int(M), int(R), VEC_KINDS[vec_kind], PRECISIONS[precision], int(col_block),
                  int(seed) % 2**64, int(lanczos_steps), float(margin), int(bool(autotune)))


def sector_dim(n_sites: int, n_up: int) -> int:
    return int(load().kpm_sector_dim(n_sites, n_up))


def sector_states(n_sites: int, n_up: int, stream=None) -> torch.Tensor:
    """Basis words in rank order (int32 tensor holding the uint32 bit patterns)."""
    dim = math.comb(n_sites, n_up)
    out = torch.empty(max(dim, 1), dtype=torch.int32, device="cuda")
    _check(load().kpm_sector_states(n_sites, n_up, _ptr(out), _stream(stream)), "kpm_sector_states")
    return out[:dim]


def sector_matrix(sector, row0: int, nrows: int, max_nb: int | None = None, stream=None):
    """(cols [nrows, max_nb] int32 (uint32 bits), bond [nrows, max_nb], cnt [nrows], diag [nrows])."""
    ps = ProblemSet([sector])
    nb = max_nb or max(1, sector.cluster.n_bonds)
    cols = torch.zeros((max(nrows, 1), nb), dtype=torch.int32, device="cuda")
    bond = torch.full((max(nrows, 1), nb), -1, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(max(nrows, 1), dtype=torch.int32, device="cuda")
    diag = torch.zeros(max(nrows, 1), dtype=torch.float64, device="cuda")
    _check(load().kpm_sector_matrix(ps.arr, row0, nrows, nb, _ptr(cols), _ptr(bond), _ptr(cnt), _ptr(diag),
                                    _stream(stream)), "kpm_sector_matrix")
    return cols[:nrows], bond[:nrows], cnt[:nrows], diag[:nrows]


def spectral_bounds(sectors, steps=50, margin=0.01, seed=0, stream=None) -> np.ndarray:
    ps = ProblemSet(sectors)
    out = (c_double * (2 * len(ps)))()
    _check(load().kpm_spectral_bounds(ps.arr, len(ps), steps, margin, seed, out, _stream(stream)),
           "kpm_spectral_bounds")
    return np.array(out[:]).reshape(len(ps), 2)


def moments_workspace_size(problems: ProblemSet, params: Params) -> int:
    return int(load().chebyshev_moments_workspace_size(problems.arr, len(problems), ctypes.byref(params)))


def chebyshev_moments(sectors, M, R=1, vec_kind="rademacher", precision="fp64", eps=0.025, seed=0,
                      col_block=0, bounds=None, lanczos_steps=50, margin=0.01, workspace=None,
                      stream=None, problems=None, autotune=False):
    """Moments mu [n, M] (float64, cuda) and (a, b) [n, 2] of Eqs. (4)-(7)."""
    ps = problems or ProblemSet(sectors, bounds)
    q = make_params(M, R, vec_kind, precision, eps, seed, col_block, lanczos_steps, margin, autotune)
    mu = torch.empty((len(ps), M), dtype=torch.float64, device="cuda")
    ab = torch.empty((len(ps), 2), dtype=torch.float64, device="cuda")
    if workspace is None:
        nbytes = moments_workspace_size(ps, q)
        if nbytes == 0:
            raise KPMError(KPM_EINVAL, "chebyshev_moments_workspace_size")
        workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    _check(load().chebyshev_moments(ps.arr, len(ps), ctypes.byref(q), _ptr(mu), _ptr(ab), _ptr(workspace),
                                    workspace.numel(), _stream(stream)), "chebyshev_moments")
    return mu, ab


def chebyshev_moments_noalloc(sectors, M, R=1, vec_kind="rademacher", precision="fp64", eps=0.025,
                              seed=0, col_block=0, bounds=None, lanczos_steps=50, margin=0.01,
                              stream=None, problems=None, out=None):
    """chebyshev_moments on the library's static per-GPU workspace (no device
    allocation inside the call).  `out` = (mu [n, M], ab [n, 2]) float64 cuda
    tensors to write into; allocated here when None."""
    ps = problems or ProblemSet(sectors, bounds)
    q = make_params(M, R, vec_kind, precision, eps, seed, col_block, lanczos_steps, margin, False)
    if out is None:
        out = (torch.empty((len(ps), M), dtype=torch.float64, device="cuda"),
               torch.empty((len(ps), 2), dtype=torch.float64, device="cuda"))
    mu, ab = out
    if mu.shape != (len(ps), M) or ab.shape != (len(ps), 2) or mu.dtype != torch.float64 \
            or ab.dtype != torch.float64 or not (mu.is_contiguous() and ab.is_contiguous()):
        raise KPMError(KPM_EINVAL, "chebyshev_moments_noalloc: out shapes")
    _check(load().chebyshev_moments_noalloc(ps.arr, len(ps), ctypes.byref(q), _ptr(mu), _ptr(ab),
                                            _stream(stream)), "chebyshev_moments_noalloc")
    return mu, ab


def chebyshev_vectors(sector, n_vec, R=1, vec_kind="rademacher", precision="fp64", eps=0.025, seed=0,
                      col_block=0, bounds=None, lanczos_steps=50, margin=0.01, stream=None):
    """v_{n_vec} of one sector, [dim, real columns] (float32 for "fp32"
    storage, else float64, cuda), and (a, b) [2]."""
    ps = ProblemSet([sector], None if bounds is None else [bounds])
    q = make_params(max(2, 2 * n_vec), R, vec_kind, precision, eps, seed, col_block, lanczos_steps, margin)
    ncols = sector.dim if vec_kind == "basis" else R * (2 if vec_kind == "complex_gaussian" else 1)
    dt = torch.float32 if precision == "fp32" else torch.float64
    out = torch.empty((sector.dim, ncols), dtype=dt, device="cuda")
    ab = torch.empty(2, dtype=torch.float64, device="cuda")
    lib = load()
    nbytes = lib.chebyshev_vectors_workspace_size(ps.arr, ctypes.byref(q), n_vec)
    if nbytes == 0:
        raise KPMError(KPM_EINVAL, "chebyshev_vectors_workspace_size")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    _check(lib.chebyshev_vectors(ps.arr, ctypes.byref(q), n_vec, _ptr(out), _ptr(ab), _ptr(ws), ws.numel(),
                                 _stream(stream)), "chebyshev_vectors")
    return out, ab


def thermo(mu, ab, sectors, T, kernel="jackson", n_nodes=0, stream=None):
    """ln Z, E, C, chi [n_clusters, n_T] and the Z <= 0 flags."""
    ps = sectors if isinstance(sectors, ProblemSet) else ProblemSet(sectors)
    mu = _f64(mu)
    ab = _f64(ab)
    T = torch.as_tensor(T, dtype=torch.float64, device="cuda").contiguous()
    nc, nT = ps.n_clusters, T.numel()
    out = {k: torch.empty((nc, nT), dtype=torch.float64, device="cuda") for k in ("lnZ", "E", "C", "chi")}
    out["z_nonpos"] = torch.empty((nc, nT), dtype=torch.uint8, device="cuda")
    _check(load().kpm_thermo(_ptr(mu), _ptr(ab), ps.arr, len(ps), mu.shape[1], KERNELS[kernel], n_nodes,
                             _ptr(T), nT, _ptr(out["lnZ"]), _ptr(out["E"]), _ptr(out["C"]), _ptr(out["chi"]),
                             _ptr(out["z_nonpos"]), _stream(stream)), "kpm_thermo")
    return out


def thermo_field(mu, ab, sectors, T, h, kernel="jackson", n_nodes=0, stream=None):
    """ln Z, E, C, chi, M = <S^z> [n_clusters, n_pts] at the points (T, h) with
    the Zeeman term h S^z (h = g mu_B B), and the Z <= 0 flags."""
    ps = sectors if isinstance(sectors, ProblemSet) else ProblemSet(sectors)
    mu = _f64(mu)
    ab = _f64(ab)
    T = torch.as_tensor(T, dtype=torch.float64, device="cuda").contiguous()
    h = torch.as_tensor(h, dtype=torch.float64, device="cuda").expand_as(T).contiguous()
    nc, nT = ps.n_clusters, T.numel()
    out = {k: torch.empty((nc, nT), dtype=torch.float64, device="cuda") for k in ("lnZ", "E", "C", "chi", "M")}
    out["z_nonpos"] = torch.empty((nc, nT), dtype=torch.uint8, device="cuda")
    _check(load().kpm_thermo_field(_ptr(mu), _ptr(ab), ps.arr, len(ps), mu.shape[1], KERNELS[kernel], n_nodes,
                                   _ptr(T), _ptr(h), nT, _ptr(out["lnZ"]), _ptr(out["E"]), _ptr(out["C"]),
                                   _ptr(out["chi"]), _ptr(out["M"]), _ptr(out["z_nonpos"]), _stream(stream)),
           "kpm_thermo_field")
    return out


def ftlm(sectors, krylov_dim, R=1, vec_kind="rademacher", T=(1.0,), h=None, seed=0, ritz=False,
         col_block=0, stream=None):
    """Finite-temperature Lanczos thermodynamics: ln Z, E, C, chi, M = <S^z>
    [n_clusters, n_pts] at the points (T, h); with ritz=True also the Ritz
    values and estimator weights [real columns, steps]."""
    ps = sectors if isinstance(sectors, ProblemSet) else ProblemSet(sectors)
    q = make_params(krylov_dim, R, vec_kind, "fp64", 0.0, seed, col_block)
    T = torch.as_tensor(T, dtype=torch.float64, device="cuda").contiguous()
    hh = None if h is None else torch.as_tensor(h, dtype=torch.float64, device="cuda").expand_as(T).contiguous()
    nc, nT = ps.n_clusters, T.numel()
    out = {k: torch.empty((nc, nT), dtype=torch.float64, device="cuda") for k in ("lnZ", "E", "C", "chi", "M")}
    lib = load()
    nbytes = lib.kpm_ftlm_workspace_size(ps.arr, len(ps), ctypes.byref(q))
    if nbytes == 0:
        raise KPMError(KPM_EINVAL, "kpm_ftlm_workspace_size")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    rz = wt = None
    if ritz:
        dims = [s.dim for s in ps.sectors]
        cols = sum(s.dim if vec_kind == "basis" else R * (2 if vec_kind == "complex_gaussian" else 1)
                   for s in ps.sectors)
        steps = max(1, min(krylov_dim, max(dims)))
        rz = torch.empty((cols, steps), dtype=torch.float64, device="cuda")
        wt = torch.empty_like(rz)
    _check(lib.kpm_ftlm(ps.arr, len(ps), ctypes.byref(q), _ptr(T), _ptr(hh), nT, _ptr(out["lnZ"]), _ptr(out["E"]),
                        _ptr(out["C"]), _ptr(out["chi"]), _ptr(out["M"]), _ptr(rz), _ptr(wt), _ptr(ws),
                        ws.numel(), _stream(stream)), "kpm_ftlm")
    if ritz:
        out["ritz"], out["weight"] = rz, wt
    return out


def sector_eigenvalues(sectors, max_dim=512, stream=None):
    """Exact spectra [n, max_dim] (ascending, NaN-padded; NaN rows for sectors
    larger than max_dim)."""
    ps = sectors if isinstance(sectors, ProblemSet) else ProblemSet(sectors)
    lib = load()
    nbytes = lib.kpm_sector_eigenvalues_workspace_size(ps.arr, len(ps), max_dim)
    if nbytes == 0:
        raise KPMError(KPM_EINVAL, "kpm_sector_eigenvalues_workspace_size")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    ev = torch.empty((len(ps), max_dim), dtype=torch.float64, device="cuda")
    _check(lib.kpm_sector_eigenvalues(ps.arr, len(ps), max_dim, _ptr(ev), _ptr(ws), ws.numel(),
                                      _stream(stream)), "kpm_sector_eigenvalues")
    return ev


def thermo_hybrid(mu, ab, sectors, evals, exact, T, h=None, kernel="jackson", n_nodes=0, stream=None):
    """Thermodynamics [n_clusters, n_pts] with the sectors flagged in `exact`
    taken from their spectra (rows of evals) and the rest from their moments."""
    ps = sectors if isinstance(sectors, ProblemSet) else ProblemSet(sectors)
    T = torch.as_tensor(T, dtype=torch.float64, device="cuda").contiguous()
    hh = None if h is None else torch.as_tensor(h, dtype=torch.float64, device="cuda").expand_as(T).contiguous()
    ex = np.ascontiguousarray(np.asarray(exact, dtype=np.uint8))
    if ex.size != len(ps):
        raise KPMError(KPM_EINVAL, "thermo_hybrid: one exact flag per problem")
    evals = _f64(evals)
    mu, ab = _f64(mu), _f64(ab)
    nc, nT = ps.n_clusters, T.numel()
    out = {k: torch.empty((nc, nT), dtype=torch.float64, device="cuda") for k in ("lnZ", "E", "C", "chi", "M")}
    out["z_nonpos"] = torch.empty((nc, nT), dtype=torch.uint8, device="cuda")
    _check(load().kpm_thermo_hybrid(_ptr(mu), _ptr(ab), ps.arr, len(ps), mu.shape[1],
                                    KERNELS[kernel], n_nodes, _ptr(evals), evals.shape[1],
                                    ex.ctypes.data_as(c_void_p), _ptr(T), _ptr(hh), nT, _ptr(out["lnZ"]),
                                    _ptr(out["E"]), _ptr(out["C"]), _ptr(out["chi"]), _ptr(out["M"]),
                                    _ptr(out["z_nonpos"]), _stream(stream)), "kpm_thermo_hybrid")
    return out


def thermo_vjp(mu, ab, sectors, T, wC, wchi, kernel="jackson", n_nodes=0, stream=None):
    """dL/dmu [n, M] for L = sum wC C + wchi chi."""
    ps = sectors if isinstance(sectors, ProblemSet) else ProblemSet(sectors)
    mu, ab = _f64(mu), _f64(ab)
    T = torch.as_tensor(T, dtype=torch.float64, device="cuda").contiguous()
    wC = torch.as_tensor(wC, dtype=torch.float64, device="cuda").contiguous()
    wchi = torch.as_tensor(wchi, dtype=torch.float64, device="cuda").contiguous()
    lam = torch.empty_like(mu)
    _check(load().kpm_thermo_vjp(_ptr(mu), _ptr(ab), ps.arr, len(ps), mu.shape[1], KERNELS[kernel],
                                 n_nodes, _ptr(T), T.numel(), _ptr(wC), _ptr(wchi), _ptr(lam), _stream(stream)),
           "kpm_thermo_vjp")
    return lam


def autotune_reset():
    _check(load().kpm_autotune_reset(), "kpm_autotune_reset")


def last_run_stats() -> dict:
    s = RunStats()
    _check(load().kpm_last_run_stats(ctypes.byref(s)), "kpm_last_run_stats")
    return {f: getattr(s, f) for f, _ in RunStats._fields_}


def moments_vjp(sectors, M, R, ab, dmu, vec_kind="rademacher", precision="fp64", eps=0.025, seed=0,
                col_block=0, ckpt_every=64, problems=None, stream=None):
    """dL/dJ (concatenated per problem, bond order) for dL/dmu = dmu, with the
    rescaling ab held fixed (same seeds and vectors as chebyshev_moments)."""
    ps = problems or ProblemSet(sectors)
    q = make_params(M, R, vec_kind, precision, eps, seed, col_block)
    lib = load()
    nbytes = lib.chebyshev_moments_vjp_workspace_size(ps.arr, len(ps), ctypes.byref(q), ckpt_every)
    if nbytes == 0:
        raise KPMError(KPM_EINVAL, "chebyshev_moments_vjp_workspace_size")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    nb = sum(s.cluster.n_bonds for s in ps.sectors)
    dJ = torch.empty(max(nb, 1), dtype=torch.float64, device="cuda")
    ab = _f64(ab)
    dmu = dmu.to(device="cuda", dtype=torch.float64).contiguous()
    _check(lib.chebyshev_moments_vjp(ps.arr, len(ps), ctypes.byref(q), _ptr(ab), _ptr(dmu), ckpt_every,
                                     _ptr(dJ), _ptr(ws), nbytes, _stream(stream)), "chebyshev_moments_vjp")
    return dJ[:nb]


def moments_ckpt(sectors, M, R=1, vec_kind="rademacher", precision="fp64", eps=0.025, seed=0,
                 col_block=0, ckpt_every=64, bounds=None, problems=None, stream=None):
    """Moments mu [n, M] and (a, b) [n, 2] as chebyshev_moments, with the
    recursion's checkpoints kept in the returned workspace for moments_vjp_resume."""
    ps = problems or ProblemSet(sectors, bounds)
    q = make_params(M, R, vec_kind, precision, eps, seed, col_block)
    lib = load()
    nbytes = lib.chebyshev_moments_ckpt_workspace_size(ps.arr, len(ps), ctypes.byref(q), ckpt_every)
    if nbytes == 0:
        raise KPMError(KPM_EINVAL, "chebyshev_moments_ckpt_workspace_size")
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    mu = torch.empty((len(ps), M), dtype=torch.float64, device="cuda")
    ab = torch.empty((len(ps), 2), dtype=torch.float64, device="cuda")
    _check(lib.chebyshev_moments_ckpt(ps.arr, len(ps), ctypes.byref(q), ckpt_every, _ptr(mu), _ptr(ab),
                                      _ptr(ws), nbytes, _stream(stream)), "chebyshev_moments_ckpt")
    return mu, ab, ws


def moments_vjp_resume(ps, M, R, ab, dmu, ws, vec_kind="rademacher", precision="fp64", eps=0.025, seed=0,
                       col_block=0, ckpt_every=64, stream=None):
    """dL/dJ from the checkpoints moments_ckpt left in ws (same arguments)."""
    q = make_params(M, R, vec_kind, precision, eps, seed, col_block)
    nb = sum(s.cluster.n_bonds for s in ps.sectors)
    dJ = torch.empty(max(nb, 1), dtype=torch.float64, device="cuda")
    dmu = dmu.to(device="cuda", dtype=torch.float64).contiguous()
    _check(load().chebyshev_moments_vjp_resume(ps.arr, len(ps), ctypes.byref(q), _ptr(_f64(ab)),
                                               _ptr(dmu), ckpt_every, _ptr(dJ), _ptr(ws), ws.numel(),
                                               _stream(stream)), "chebyshev_moments_vjp_resume")
    return dJ[:nb]


def cluster_bond_grad(problems, dJ, stream=None):
    """Per-cluster dL/dJ (clusters by id, bonds in order) from the per-problem
    derivatives dJ (problem after problem), summed by the library."""
    ps = problems if isinstance(problems, ProblemSet) else ProblemSet(problems)
    ncl = max(s.cluster_id for s in ps.sectors) + 1
    nb = [0] * ncl
    for s in ps.sectors:
        nb[s.cluster_id] = s.cluster.n_bonds
    out = torch.empty(max(sum(nb), 1), dtype=torch.float64, device="cuda")
    dJ = dJ.to(device="cuda", dtype=torch.float64).contiguous()
    _check(load().kpm_cluster_bond_grad(ps.arr, len(ps), _ptr(dJ), _ptr(out), _stream(stream)),
           "kpm_cluster_bond_grad")
    return out[:sum(nb)]


def thermo_grad(sectors, M, R, T, wC, wchi, vec_kind="rademacher", precision="fp64", eps=0.025, seed=0,
                col_block=0, kernel="none", n_nodes=0, ckpt_every=64, bounds=None, problems=None,
                stream=None):
    """L = sum wC C + wchi chi and dL/dJ (per problem, bond order), bounds fixed."""
    ps = problems or ProblemSet(sectors, bounds)
    q = make_params(M, R, vec_kind, precision, eps, seed, col_block)
    T = torch.as_tensor(T, dtype=torch.float64, device="cuda").contiguous()
    wC = torch.as_tensor(wC, dtype=torch.float64, device="cuda").contiguous()
    wchi = torch.as_tensor(wchi, dtype=torch.float64, device="cuda").contiguous()
    nb = sum(s.cluster.n_bonds for s in ps.sectors)
    L = torch.empty(1, dtype=torch.float64, device="cuda")
    dJ = torch.empty(max(nb, 1), dtype=torch.float64, device="cuda")
    ab = torch.empty((len(ps), 2), dtype=torch.float64, device="cuda")
    _check(load().kpm_thermo_grad(ps.arr, len(ps), ctypes.byref(q), KERNELS[kernel], n_nodes, _ptr(T),
                                  T.numel(), _ptr(wC), _ptr(wchi), ckpt_every, _ptr(L), _ptr(dJ), _ptr(ab),
                                  None, 0, _stream(stream)), "kpm_thermo_grad")
    return L[0], dJ[:nb], ab


class KPMMoments(torch.autograd.Function):
    """mu, ab = KPMMoments.apply(J, cluster, n_ups, M, R, vec_kind, precision, eps, seed, col_block,
    bounds, ckpt_every): Chebyshev moments of the sectors n_ups of one cluster whose
    couplings are J (float64 tensor [n_bonds]); backward gives dL/dJ through the
    recursion adjoint with the rescaling held at the forward's values.  The
    forward keeps the recursion's checkpoints (one workspace held until
    backward), so the backward runs only the reverse sweep."""

    @staticmethod
    def forward(ctx, J, cluster, n_ups, M, R, vec_kind="rademacher", precision="fp64", eps=0.025, seed=0,
                col_block=0, bounds=None, ckpt_every=64):
        import workloads as W
        cl = cluster.with_J(J.detach().to("cpu", torch.float64).numpy())
        secs = [W.Sector(cl, k, 0) for k in n_ups]
        ps = ProblemSet(secs, bounds)
        mu, ab, ws = moments_ckpt(None, M, R, vec_kind, precision, eps, seed, col_block, ckpt_every, problems=ps)
        ctx.ps, ctx.ab, ctx.ws = ps, ab, ws
        ctx.args = (M, R, vec_kind, precision, eps, seed, col_block, ckpt_every)
        ctx.n_bonds, ctx.J_device = cl.n_bonds, J.device
        ctx.mark_non_differentiable(ab)
        return mu, ab

    @staticmethod
    def backward(ctx, dmu, dab):
        M, R, vec_kind, precision, eps, seed, col_block, ckpt_every = ctx.args
        dJ = moments_vjp_resume(ctx.ps, M, R, ctx.ab, dmu, ctx.ws, vec_kind, precision, eps, seed, col_block,
                                ckpt_every)
        ctx.ws = None
        dJ = cluster_bond_grad(ctx.ps, dJ).to(ctx.J_device)
        return (dJ,) + (None,) * 11


class KPMThermo(torch.autograd.Function):
    """C, chi = KPMThermo.apply(mu, ab, problems, T, kernel, n_nodes) for one
    or more clusters ([n_clusters, n_T]); backward gives dL/dmu."""

    @staticmethod
    def forward(ctx, mu, ab, problems, T, kernel="none", n_nodes=0):
        out = thermo(mu, ab, problems, T, kernel, n_nodes)
        ctx.save_for_backward(mu, ab)
        ctx.problems, ctx.T, ctx.kernel, ctx.n_nodes = problems, T, kernel, n_nodes
        return out["C"], out["chi"]

    @staticmethod
    def backward(ctx, dC, dchi):
        mu, ab = ctx.saved_tensors
        ps = ctx.problems if isinstance(ctx.problems, ProblemSet) else ProblemSet(ctx.problems)
        shape = (ps.n_clusters, torch.as_tensor(ctx.T).numel())
        zero = torch.zeros(shape, dtype=torch.float64, device="cuda")
        wC = zero if dC is None else dC.contiguous()
        wchi = zero if dchi is None else dchi.contiguous()
        lam = thermo_vjp(mu, ab, ps, ctx.T, wC, wchi, ctx.kernel, ctx.n_nodes)
        return lam, None, None, None, None, None
