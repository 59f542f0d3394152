"""Every step kernel (column-chunk, row, block, block-table, slice) against the oracle on the same
seeds and bounds, including block geometries that force many small tiles,
several blocks per tile and clusters smaller than the block width.

Tolerances as in the moments tests: |mu_gpu - mu_oracle| <= tol * mu_0 with
tol = 1e-10 (float64 vectors) and 1e-5 (float32 storage)."""
import functools

import numpy as np
import pytest

import workloads as W
from oracle import hamiltonian, moments

pytestmark = pytest.mark.gpu

KERNELS = {
    "chunk": ({"KPM_BLOCK": "0", "KPM_ROW_KERNEL": "0"}, 0),
    "row": ({"KPM_BLOCK": "0", "KPM_ROW_KERNEL": "1"}, None),
    "block": ({"KPM_BLOCK": "1"}, 2),
    # 64-row sub-tiles (low words of 7 bits), at most 2 blocks per tile, 3
    # sub-tiles per workgroup, 8 gathers in flight
    "block_small": ({"KPM_BLOCK": "1", "KPM_BLOCK_ROWS": "64", "KPM_BLOCK_MAX": "2",
                     "KPM_SUB_PER_TILE": "3", "KPM_GATHER_BATCH": "8"}, 2),
    # 4 low bits: most bonds are high-high or mixed
    "block_l4": ({"KPM_BLOCK": "1", "KPM_BLOCK_L": "4", "KPM_SUB_PER_TILE": "1"}, 2),
    # block-table kernel, default geometry, small tiles and 4 low bits
    "tab": ({"KPM_BLOCK": "2"}, 3),
    "tab_small": ({"KPM_BLOCK": "2", "KPM_BLOCK_ROWS": "64", "KPM_BLOCK_MAX": "2",
                   "KPM_SUB_PER_TILE": "3", "KPM_GATHER_BATCH": "8"}, 3),
    "tab_l4": ({"KPM_BLOCK": "2", "KPM_BLOCK_L": "4", "KPM_SUB_PER_TILE": "1"}, 3),
    # slice kernel (each wave on rows of one block): default geometry, small
    # sub-tiles with 4 high-high rows per batch, 4 low bits, 10 low bits
    "slice": ({"KPM_BLOCK": "3"}, 5),
    "slice_small": ({"KPM_BLOCK": "3", "KPM_BLOCK_ROWS": "64", "KPM_BLOCK_MAX": "2",
                     "KPM_SUB_PER_TILE": "3", "KPM_GATHER_BATCH": "4"}, 5),
    "slice_l4": ({"KPM_BLOCK": "3", "KPM_BLOCK_L": "4", "KPM_SUB_PER_TILE": "1"}, 5),
    "slice_l10": ({"KPM_BLOCK": "3", "KPM_BLOCK_L": "10", "KPM_SUB_PER_TILE": "2"}, 5),
    # contiguous tile ranges per XCD in place of the default per-column-block chunks
    "slice_contig": ({"KPM_BLOCK": "3", "KPM_XCD_REMAP": "1"}, 5),
    # waves per tile (default 2 where rows are 16-byte multiples): one wave,
    # four waves, four waves on tiles of many small blocks (slices numbered
    # across blocks), two waves on 4-bit blocks (one slice per block, so a
    # wave skips every other block)
    "slice_w1": ({"KPM_BLOCK": "3", "KPM_SLICE_WAVES": "1"}, 5),
    "slice_w4": ({"KPM_BLOCK": "3", "KPM_SLICE_WAVES": "4"}, 5),
    "slice_w4_small": ({"KPM_BLOCK": "3", "KPM_SLICE_WAVES": "4", "KPM_BLOCK_ROWS": "64", "KPM_BLOCK_MAX": "2",
                        "KPM_SUB_PER_TILE": "3"}, 5),
    "slice_w2_l4": ({"KPM_BLOCK": "3", "KPM_SLICE_WAVES": "2", "KPM_BLOCK_L": "4", "KPM_SUB_PER_TILE": "2"}, 5),
}


_BOUNDS = {}


def _bounds(sec):
    key = (id(sec.cluster), sec.n_up)
    if key in _BOUNDS:
        return _BOUNDS[key][1:]
    H = hamiltonian.sector_hamiltonian(sec.cluster, sec.n_up)
    if H.shape[0] <= 1000:
        e = np.linalg.eigvalsh(H.toarray())
        lo, hi = e.min(), e.max()
    else:
        lo, hi = moments.spectral_bounds(sec, 80, 0.02, 0, H=H)
    if hi - lo < 1e-8:
        lo, hi = lo - 0.5, hi + 0.5
    _BOUNDS[key] = (sec.cluster, (lo, hi), H)   # the cluster keeps its id valid
    return (lo, hi), H


def _check(kpm, monkeypatch, kernel, secs, M, R, kind, precision, col_block, seed=0, eps=0.025):
    env, kid = KERNELS[kernel]
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    bl, Hs = zip(*[_bounds(s) for s in secs])
    mu, _ = kpm.chebyshev_moments(secs, M, R, kind, precision, eps, seed, col_block, bounds=list(bl))
    st = kpm.last_run_stats()
    if kid is not None:
        assert st["kernel"] == kid, st
    mu = mu.cpu().numpy()
    tol = 1e-10 if precision == "fp64" else 1e-5
    for p, (s, (lo, hi), H) in enumerate(zip(secs, bl, Hs)):
        a, b = hamiltonian.scale_from_bounds(lo, hi, eps)
        want = moments.sector_moments(s, a, b, M, R, kind, seed, H=H)
        err = np.abs(mu[p] - want).max() / abs(want[0])
        assert err <= tol, (kernel, p, s.n_up, err)
    return mu


@functools.lru_cache(None)
def _batched():
    secs = []
    for cid, cl in enumerate([W.ring(8), W.random_regular_cluster(11, 3, 2, J_range=(0.5, 1.5)),
                              W.j1j2_chain(14, 1.0, 0.5), W.ladder(12)]):
        secs += W.sectors(cl, cluster_id=cid)
    return tuple(secs)


@pytest.mark.parametrize("kernel", list(KERNELS))
@pytest.mark.parametrize("precision,kind,R,col_block", [
    ("fp64", "rademacher", 5, 0), ("fp64", "complex_gaussian", 3, 4), ("fp32", "rademacher", 12, 0),
    ("fp32", "complex_gaussian", 10, 20)])
def test_batched_all_sectors(kpm, monkeypatch, kernel, precision, kind, R, col_block):
    """Four clusters (N = 8, 11, 14, 12), all S^z >= 0 sectors, one call."""
    _check(kpm, monkeypatch, kernel, list(_batched()), 48, R, kind, precision, col_block, seed=4)


@pytest.mark.parametrize("kernel", list(KERNELS))
def test_j1j2_n18_sz0_wide_block(kpm, monkeypatch, kernel):
    """N=18 J1-J2 chain S^z=0 (48,620 states: hundreds of tiles), 20 float32
    columns in one block."""
    secs = W.sectors(W.j1j2_chain(18, 1.0, 0.5), only_sz0=True)
    _check(kpm, monkeypatch, kernel, secs, 40, 10, "complex_gaussian", "fp32", 20, seed=2)


@pytest.mark.parametrize("kernel", ["block", "block_small", "block_l4", "tab", "tab_small", "tab_l4", "slice",
                                    "slice_small", "slice_l4", "slice_l10", "slice_w1", "slice_w4", "slice_w2_l4"])
def test_block_extreme_sectors(kpm, monkeypatch, kernel):
    """Sectors whose blocks are tiny (n_up near N) or single (N below the
    block width), dimension-1 sectors and the dimer."""
    cl = W.ring(16)
    secs = [W.Sector(cl, k, 0) for k in (16, 15, 14, 13)] + W.sectors(W.ring(5), cluster_id=1)
    secs += [W.Sector(W.dimer(), 1, 2), W.Sector(W.dimer(), 2, 2)]
    for prec in ("fp64", "fp32"):
        _check(kpm, monkeypatch, kernel, secs, 24, 3, "rademacher", prec, 0, seed=9)


def test_kernels_agree_ring20(kpm, monkeypatch):
    """Ring N=20 S^z=0 (184,756 states), float64, 8 columns: every kernel's
    moments agree to rounding (they sum the bonds in different orders)."""
    secs = W.sectors(W.ring(20), only_sz0=True)
    bl = [(-9.2, 5.1)]
    out = {}
    for name, (env, _) in KERNELS.items():
        with monkeypatch.context() as m:
            for k, v in env.items():
                m.setenv(k, v)
            mu, _ = kpm.chebyshev_moments(secs, 200, 8, "rademacher", "fp64", 0.025, 1, 8, bounds=bl)
            out[name] = mu.cpu().numpy()[0]
    ref = out["chunk"]
    for name, mu in out.items():
        assert np.abs(mu - ref).max() <= 1e-11 * ref[0], name


def test_slice_workgroup_mappings_identical(kpm, monkeypatch):
    """The slice kernel's workgroup-to-tile maps (per-column-block chunks per
    XCD, with idle workgroups where a block's tile count is not a multiple of
    8, and contiguous ranges) run the same tiles: bit-identical moments on a
    batch of many problems and column blocks."""
    secs = list(_batched()) + W.sectors(W.ring(18), only_sz0=True)
    bl = [_bounds(s)[0] for s in secs]
    monkeypatch.setenv("KPM_BLOCK", "3")
    out = {}
    for remap in ("1", "2"):
        monkeypatch.setenv("KPM_XCD_REMAP", remap)
        mu, _ = kpm.chebyshev_moments(secs, 64, 10, "complex_gaussian", "fp32", 0.025, 6, 4, bounds=bl)
        assert kpm.last_run_stats()["kernel"] == 5
        out[remap] = mu.cpu().numpy()
    assert np.array_equal(out["1"], out["2"])


@pytest.mark.parametrize("precision,col_block,env_waves,want", [
    ("fp32", 4, None, 2), ("fp32", 8, "4", 4), ("fp32", 4, "1", 1), ("fp64", 2, None, 2),
    ("fp32", 2, None, 1), ("fp64", 1, "4", 1), ("fp32r", 4, None, 2), ("fp32r", 4, "4", 4),
    ("fp32r", 2, "1", 1)])
def test_slice_waves_per_tile(kpm, monkeypatch, precision, col_block, env_waves, want):
    """Waves per workgroup as planned: 2 by default, as asked where rows are
    16 or 32 bytes (float32 blocks of 4 or 8 columns, float64 blocks of 2)
    and for float32 + residual storage (rows decoded through registers), 1
    for narrower plain rows; the moments match the oracle either way."""
    monkeypatch.setenv("KPM_BLOCK", "3")
    if env_waves:
        monkeypatch.setenv("KPM_SLICE_WAVES", env_waves)
    secs = W.sectors(W.ring(16), only_sz0=True)
    (lo, hi), H = _bounds(secs[0])
    mu, _ = kpm.chebyshev_moments(secs, 40, 8, "rademacher", precision, 0.025, 5, col_block, bounds=[(lo, hi)])
    st = kpm.last_run_stats()
    assert st["kernel"] == 5 and st["waves"] == want, st
    a, b = hamiltonian.scale_from_bounds(lo, hi, 0.025)
    ref = moments.sector_moments(secs[0], a, b, 40, 8, "rademacher", 5, H=H,
                                 store=moments.F32R if precision == "fp32r" else np.float64)
    tol = {"fp64": 1e-10, "fp32": 1e-5, "fp32r": 1e-10}[precision]
    assert np.abs(mu.cpu().numpy()[0] - ref).max() <= tol * abs(ref[0])


# ------------------------------------------------- relabelled sites (block kernels)

def _rr(n, seed):
    return W.random_regular_cluster(n, 3, seed, J_range=(0.5, 1.5))


@pytest.mark.parametrize("kernel", ["block", "tab", "tab_small", "slice", "slice_small"])
@pytest.mark.parametrize("kind,R", [("rademacher", 4), ("gaussian", 3), ("complex_gaussian", 2), ("basis", 1)])
def test_relabelled_random_graphs(kpm, monkeypatch, kernel, kind, R):
    """Random 3-regular clusters (N = 13, 15) whose labels cut many bonds at
    the low/high boundary: the block kernels relabel their sites, and the
    moments still match the oracle (start vectors drawn by original rank)."""
    secs = W.sectors(_rr(13, 21), cluster_id=0) + W.sectors(_rr(15, 22), cluster_id=1)
    if kind == "basis":
        secs = [s for s in secs if s.dim <= 500]
    _check(kpm, monkeypatch, kernel, secs, 32, R, kind, "fp64", 0, seed=3)
    assert kpm.last_run_stats()["relabelled"] == len(secs)


def test_relabelling_keeps_the_ring(kpm, monkeypatch):
    monkeypatch.setenv("KPM_BLOCK", "2")
    kpm.chebyshev_moments(W.sectors(W.ring(16), only_sz0=True), 8, 2, "rademacher", "fp64", bounds=[(-8, 5)])
    assert kpm.last_run_stats()["relabelled"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_relabelled_vectors_in_original_order(kpm, monkeypatch, precision):
    """v_3 of a relabelled N=18 sector, exported in the original rank order,
    against the oracle's dense recursion."""
    from oracle import rows
    monkeypatch.setenv("KPM_BLOCK", "2")
    s = W.sectors(_rr(18, 23), only_sz0=True)[0]
    (lo, hi), H = _bounds(s)
    kpm.chebyshev_moments([s], 8, 4, "gaussian", precision, 0.025, 5, 4, bounds=[(lo, hi)])
    assert kpm.last_run_stats()["relabelled"] == 1          # the same plan as the vectors'
    V, _ = kpm.chebyshev_vectors(s, 3, 4, "gaussian", precision, 0.025, 5, 4, bounds=(lo, hi))
    a, b = hamiltonian.scale_from_bounds(lo, hi, 0.025)
    sample = np.concatenate([np.random.default_rng(0).choice(s.dim, 40, replace=False), [0, s.dim - 1]])
    got = V.double().cpu().numpy()[sample]
    want = rows.recursion_rows(s.cluster, s.n_up, a, b, "gaussian", 5, 4, sample, 3,
                               store=np.float32 if precision == "fp32" else np.float64)
    tol = 1e-6 if precision == "fp32" else 1e-12
    assert np.abs(got - want).max() <= tol * np.abs(want).max()


def test_relabelled_lanczos_and_ftlm(kpm, monkeypatch):
    """Lanczos bounds and FTLM Ritz values through the relabelled block-table
    kernel (their start vectors come from the same original-rank draw)."""
    from oracle import ftlm
    monkeypatch.setenv("KPM_BLOCK", "2")
    secs = W.sectors(_rr(14, 24))
    got = kpm.spectral_bounds(secs, 30, 0.01, 2)
    for p, s in enumerate(secs):
        want = moments.spectral_bounds(s, 30, 0.01, 2)
        assert np.abs(got[p] - np.array(want)).max() <= 1e-9 * max(1.0, np.abs(want).max()), p
    out = kpm.ftlm(secs, 8, 2, "rademacher", T=[1.0], seed=7, ritz=True, col_block=2)
    rz = out["ritz"].cpu().numpy()
    c = 0
    for s in secs:
        for e_ref, _ in ftlm.sector_ritz(s, 8, 2, "rademacher", 7):
            e = np.sort(rz[c, :e_ref.size])
            assert np.abs(e - e_ref).max() <= 1e-9 * max(1.0, np.abs(e_ref).max()), (s.n_up, c)
            c += 1
