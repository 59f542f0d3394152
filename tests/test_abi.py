"""The C-ABI library loads, exports every function include/kpm.h declares, and
rejects invalid arguments before touching a device (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kpm.h")


def _lib_path():
    from paper_2104_13218_amd import kpm
    if not os.path.exists(kpm.LIB_PATH):
        from paper_2104_13218_amd import build
        build.build()
    return kpm.LIB_PATH


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|size_t|uint64_t|char\s*\*|char)\s*\*?\s*(\w+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_three_entry_points():
    names = declared_functions()
    for n in ("chebyshev_moments", "kpm_thermo", "kpm_thermo_grad"):
        assert n in names
    assert len(names) >= 12


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.fixture(scope="module")
def kpmlib():
    _lib_path()
    from paper_2104_13218_amd import kpm
    return kpm


def test_strerror_and_dims(kpmlib):
    assert kpmlib.strerror(0) == "ok"
    assert "bounds" in kpmlib.strerror(kpmlib.KPM_EBOUNDS)
    assert kpmlib.sector_dim(24, 12) == 2704156
    assert kpmlib.sector_dim(30, 15) == 155117520
    assert kpmlib.sector_dim(32, 16) == math.comb(32, 16)
    assert kpmlib.sector_dim(5, 7) == 0


def _problem(kpmlib, N=6, n_up=3, bonds=((0, 1), (1, 2)), J=(1.0, 1.0), cluster=0):
    import workloads as W
    bi = np.array([b[0] for b in bonds]); bj = np.array([b[1] for b in bonds])
    return kpmlib.ProblemSet([W.Sector(W.Cluster(N, bi, bj, np.array(J, float)), n_up, cluster)])


def _moments_rc(kpmlib, ps, **kw):
    q = kpmlib.make_params(**{"M": 16, "R": 2, **kw})
    lib = kpmlib.load()
    return lib.chebyshev_moments(ps.arr, len(ps), ctypes.byref(q), None, None, None, 0, None)


def test_invalid_arguments_rejected_on_host(kpmlib):
    E = kpmlib.KPM_EINVAL
    assert _moments_rc(kpmlib, _problem(kpmlib, bonds=((1, 1),), J=(1.0,))) == E        # i == j
    assert _moments_rc(kpmlib, _problem(kpmlib, bonds=((0, 6),), J=(1.0,))) == E        # site out of range
    assert _moments_rc(kpmlib, _problem(kpmlib, J=(1.0, float("nan")))) == E           # non-finite J
    assert _moments_rc(kpmlib, _problem(kpmlib, n_up=2)) == E                           # S^z < 0
    assert _moments_rc(kpmlib, _problem(kpmlib), M=1) == E
    assert _moments_rc(kpmlib, _problem(kpmlib), R=0) == E
    assert _moments_rc(kpmlib, _problem(kpmlib), eps=1.0) == E
    assert _moments_rc(kpmlib, _problem(kpmlib), col_block=65) == E
    ps = _problem(kpmlib)
    ps.arr[0].e_lo, ps.arr[0].e_hi = 1.0, 0.5                                           # empty window
    assert _moments_rc(kpmlib, ps) == E
    lib = kpmlib.load()
    q = kpmlib.make_params(M=16, R=2)
    assert lib.chebyshev_moments_workspace_size(_problem(kpmlib, n_up=1).arr, 1, ctypes.byref(q)) == 0
    assert lib.kpm_sector_states(33, 3, None, None) == E
    assert lib.kpm_sector_states(8, 9, None, None) == E


def test_workspace_size_query_is_host_only(kpmlib):
    import workloads as W
    ps = kpmlib.ProblemSet(W.sectors(W.ring(12)))
    q = kpmlib.make_params(M=256, R=20)
    n = kpmlib.load().chebyshev_moments_workspace_size(ps.arr, len(ps), ctypes.byref(q))
    # at least the two float64 recursion buffers of every (sector, column block)
    assert n >= 2 * 8 * 20 * 2**12 // 2


def test_exact_spectra_arguments_on_host(kpmlib):
    """kpm_sector_eigenvalues: workspace query and argument checks need no device."""
    import workloads as W
    lib = kpmlib.load()
    ps = kpmlib.ProblemSet(W.sectors(W.ring(12)))               # dims 924, 792, 495, 220, 66, 12, 1
    assert lib.kpm_sector_eigenvalues_workspace_size(ps.arr, len(ps), 0) == 0
    assert lib.kpm_sector_eigenvalues_workspace_size(ps.arr, len(ps), 1025) == 0
    small = lib.kpm_sector_eigenvalues_workspace_size(ps.arr, len(ps), 100)
    big = lib.kpm_sector_eigenvalues_workspace_size(ps.arr, len(ps), 1000)
    assert small >= 8 * (66**2 + 12**2 + 1) and big >= 8 * sum(d * d for d in (924, 792, 495, 220, 66, 12, 1))
    assert lib.kpm_sector_eigenvalues(ps.arr, len(ps), 2000, None, None, 0, None) == kpmlib.KPM_EINVAL
    assert lib.kpm_sector_eigenvalues(ps.arr, len(ps), 100, None, None, 0, None) == kpmlib.KPM_EINVAL


def test_empty_and_spin_arguments_on_host(kpmlib):
    """No problems, and spin-s problems outside the supported range, are
    refused before any device work; valid spin-s problems size a workspace."""
    import workloads as W
    lib = kpmlib.load()
    E = kpmlib.KPM_EINVAL
    q = kpmlib.make_params(M=16, R=2)
    ps = kpmlib.ProblemSet(W.sectors(W.ring(6)))
    assert lib.chebyshev_moments_workspace_size(ps.arr, 0, ctypes.byref(q)) == 0
    assert lib.chebyshev_moments(ps.arr, 0, ctypes.byref(q), None, None, None, 0, None) == E
    spin = kpmlib.ProblemSet(W.spin_sectors(W.ring(4), 5))
    assert lib.chebyshev_moments_workspace_size(spin.arr, len(spin), ctypes.byref(q)) > 0
    for field, value in (("two_s", 8), ("two_s", -1), ("reserved", 1)):
        bad = kpmlib.ProblemSet(W.spin_sectors(W.ring(4), 5))
        setattr(bad.arr[0], field, value)
        assert lib.chebyshev_moments_workspace_size(bad.arr, len(bad), ctypes.byref(q)) == 0, field
        assert lib.chebyshev_moments(bad.arr, len(bad), ctypes.byref(q), None, None, None, 0, None) == E
    big = kpmlib.ProblemSet([W.SpinSector(W.ring(17), 2, 17)])          # spin 1, N = 17 > 16
    assert lib.chebyshev_moments_workspace_size(big.arr, 1, ctypes.byref(q)) == 0
    low = kpmlib.ProblemSet([W.SpinSector(W.ring(4), 5, 9)])            # S^z = 9 - 10 < 0
    assert lib.chebyshev_moments_workspace_size(low.arr, 1, ctypes.byref(q)) == 0


def _top_cost(cluster, labels, L):
    """Bonds touching the top t labels, summed over t = 1 .. n - L - 1."""
    n = cluster.n_sites
    lab = np.asarray(labels)
    bi, bj = lab[np.asarray(cluster.bond_i)], lab[np.asarray(cluster.bond_j)]
    hi = np.maximum(bi, bj)
    return int(sum(np.sum(hi >= n - t) for t in range(1, n - L)))


def _cut(cluster, labels, L):
    low = np.asarray(labels)[np.asarray(cluster.bond_i)] < L
    return int(np.sum(low != (np.asarray(labels)[np.asarray(cluster.bond_j)] < L)))


@pytest.mark.parametrize("n,seed,L", [(13, 21, 9), (18, 23, 9), (24, 5, 9), (16, 2, 6), (30, 0, 9)])
def test_site_relabel_cuts_fewer_bonds(kpmlib, n, seed, L):
    """The relabelling of the block kernels (host logic): a permutation of the
    sites whose first L labels cut no more bonds than the identity's, within 2
    of the minimum over all L-sets (brute force, small n), and whose high
    labels are ordered so that no more bonds touch the top t labels, summed
    over t, than in the identity's order."""
    import itertools
    import workloads as W
    cl = W.random_regular_cluster(n, 3 if n != 30 else 4, seed)
    ps = kpmlib.ProblemSet([W.Sector(cl, (n + 1) // 2, 0)])
    perm = (ctypes.c_int32 * n)()
    rc = kpmlib.load().kpm_site_relabel(ps.arr, L, perm)
    assert rc in (0, 1), rc
    perm = np.array(perm[:])
    assert sorted(perm) == list(range(n))
    ident = _cut(cl, np.arange(n), L)
    assert _cut(cl, perm, L) <= ident
    assert (rc == 1) == (not np.array_equal(perm, np.arange(n)))
    assert _top_cost(cl, perm, L) <= _top_cost(cl, np.arange(n), L) or _cut(cl, perm, L) < ident
    if n <= 18:
        best = min(_cut(cl, [0 if i in S else L for i in range(n)], L)
                   for S in map(set, itertools.combinations(range(n), L)))
        assert _cut(cl, perm, L) <= best + 2


def test_site_relabel_keeps_the_ring(kpmlib):
    import workloads as W
    ps = kpmlib.ProblemSet([W.Sector(W.ring(24), 12, 0)])
    perm = (ctypes.c_int32 * 24)()
    assert kpmlib.load().kpm_site_relabel(ps.arr, 9, perm) == 0
    assert list(perm) == list(range(24))


def test_site_relabel_scrambled_ring(kpmlib):
    """A 24-site ring under a random labelling: the relabelling finds a set of
    9 sites cutting the minimum of 2 bonds (an arc) and orders the other 15 so
    that the top t labels touch t + 1 bonds (the minimum for t sites of a
    ring: an arc), i.e. a summed cost of 2 + 3 + ... + 15 = 119."""
    import workloads as W
    rng = np.random.default_rng(11)
    pi = rng.permutation(24)
    i = np.arange(24)
    cl = W.Cluster(24, pi[i], pi[(i + 1) % 24], np.ones(24), name="ring24_scrambled")
    ps = kpmlib.ProblemSet([W.Sector(cl, 12, 0)])
    perm = (ctypes.c_int32 * 24)()
    assert kpmlib.load().kpm_site_relabel(ps.arr, 9, perm) == 1
    perm = np.array(perm[:])
    assert sorted(perm) == list(range(24))
    assert _cut(cl, perm, 9) == 2
    assert _top_cost(cl, perm, 9) == 119 == _top_cost(W.ring(24), np.arange(24), 9)


def test_site_relabel_orders_high_sites_for_locality(kpmlib):
    """The 30-site random 4-regular cluster: the high labels are ordered so
    that fewer bonds touch the top labels than in breadth-first order from
    the low set (the order used before the locality pass; recomputed here)."""
    import workloads as W
    cl = W.random_regular_cluster(30, 4, 0)
    ps = kpmlib.ProblemSet([W.Sector(cl, 15, 0)])
    perm = (ctypes.c_int32 * 30)()
    assert kpmlib.load().kpm_site_relabel(ps.arr, 9, perm) == 1
    perm = np.array(perm[:])
    low = [v for v in range(30) if perm[v] < 9]
    adj = [[] for _ in range(30)]
    for a, b in zip(cl.bond_i, cl.bond_j):
        adj[a].append(b)
        adj[b].append(a)
    bfs, seen = [], set(low)
    queue = list(low)
    for v in queue:
        for u in sorted(adj[v]):
            if u not in seen:
                seen.add(u)
                bfs.append(u)
                queue.append(u)
    bfs += [v for v in range(30) if v not in seen]
    ref = np.empty(30, dtype=np.int64)
    for k, v in enumerate(sorted(low)):
        ref[v] = k
    for k, v in enumerate(bfs):
        ref[v] = 9 + k
    assert _cut(cl, perm, 9) == _cut(cl, ref, 9)
    assert _top_cost(cl, perm, 9) < _top_cost(cl, ref, 9)


def test_cluster_bond_grad_rejects_mixed_bond_lists(kpmlib):
    """kpm_cluster_bond_grad sums per-sector derivatives of one bond list per
    cluster: two problems of one cluster with different bond counts, or NULL
    arrays, are refused before any device work."""
    import workloads as W
    bi, bj = np.array([0, 1]), np.array([1, 2])
    c2 = W.Cluster(6, bi, bj, np.array([1.0, 1.0]))
    c1 = W.Cluster(6, bi[:1], bj[:1], np.array([1.0]))
    mixed = kpmlib.ProblemSet([W.Sector(c2, 3, 0), W.Sector(c1, 4, 0)])
    lib = kpmlib.load()
    dummy = ctypes.c_void_p(16)        # never dereferenced: the call fails on the host
    assert lib.kpm_cluster_bond_grad(mixed.arr, len(mixed), dummy, dummy, None) == kpmlib.KPM_EINVAL
    ok = kpmlib.ProblemSet([W.Sector(c2, 3, 0), W.Sector(c2, 4, 0)])
    assert lib.kpm_cluster_bond_grad(ok.arr, len(ok), None, dummy, None) == kpmlib.KPM_EINVAL


def test_noalloc_rejections_on_host(kpmlib):
    """chebyshev_moments_noalloc checks its arguments and its size limit before
    any HIP call: autotune is refused, and a call whose workspace exceeds
    KPM_NOALLOC_MAX_BYTES is KPM_ETOOLARGE."""
    import workloads as W
    lib = kpmlib.load()
    assert lib.kpm_strerror(kpmlib.KPM_ETOOLARGE).decode().startswith("needs more scratch")
    small = _problem(kpmlib)
    q = kpmlib.make_params(M=16, R=2)
    assert lib.chebyshev_moments_noalloc(small.arr, 1, ctypes.byref(q), None, None, None) == kpmlib.KPM_EINVAL
    q_tuned = kpmlib.make_params(M=16, R=2, autotune=True)
    dummy = ctypes.c_void_p(16)   # never dereferenced: rejected before any device work
    assert lib.chebyshev_moments_noalloc(small.arr, 1, ctypes.byref(q_tuned), dummy, None,
                                         None) == kpmlib.KPM_EINVAL
    big = kpmlib.ProblemSet([s for s in W.sectors(W.ring(22)) if 2 * s.n_up == 22])
    q_big = kpmlib.make_params(M=64, R=10, vec_kind="complex_gaussian")
    need = lib.chebyshev_moments_workspace_size(big.arr, 1, ctypes.byref(q_big))
    assert need > kpmlib.NOALLOC_MAX_BYTES
    assert lib.chebyshev_moments_noalloc(big.arr, 1, ctypes.byref(q_big), dummy, None,
                                         None) == kpmlib.KPM_ETOOLARGE
