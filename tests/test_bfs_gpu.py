"""Parity of the device breadth-first search (lscan_bfs) with the oracle.

Levels are unique, so they are compared exactly with the oracle's FIFO
search.  The parents are not unique (any discoverer at the level above is
right), so they are checked for validity: the source is its own parent, every
other reached vertex has a parent one level up with an edge to it, and
unreached vertices have none.  The statistics are checked against what the
levels fix: the depth, the number reached and the out-degrees of the reached
vertices."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import log
from paper_1604_04815_amd import workloads as w

pytestmark = pytest.mark.gpu


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda")


def run(gpu_lib, row, col, src, params=None, with_parents=True):
    rd, cd = dev(row, np.int64), dev(col, np.int32)
    levels, parents, stats = gpu_lib.bfs(rd, cd, src, parents=with_parents, params=params)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    return (levels.cpu().numpy(), None if parents is None else parents.cpu().numpy(),
            stats.cpu().numpy())


def has_edge(row, col, u, v):
    """Does the graph hold the edge u[k] -> v[k], for each k (binary search
    in the (row, column) keys of all edges)."""
    nv = row.shape[0] - 1
    keys = np.repeat(np.arange(nv, dtype=np.int64), np.diff(row)) * nv + col.astype(np.int64)
    if not np.all(keys[1:] >= keys[:-1]):
        keys = np.sort(keys)
    q = u.astype(np.int64) * nv + v.astype(np.int64)
    if keys.shape[0] == 0:
        return np.zeros(q.shape[0], dtype=bool)
    i = np.minimum(np.searchsorted(keys, q), keys.shape[0] - 1)
    return keys[i] == q


def check(row, col, src, levels, parents, stats, what, bad_entries=0):
    nv = row.shape[0] - 1
    want_levels = oracle.bfs_levels(row, col, src)
    if not np.array_equal(levels, want_levels):
        bad = np.flatnonzero(levels != want_levels)
        raise AssertionError(f"{what}: {bad.size} level mismatches, first at {bad[:8].tolist()}: "
                             f"got {levels[bad[:4]].tolist()} want {want_levels[bad[:4]].tolist()}")
    reached = want_levels >= 0
    deg = np.diff(row)
    assert int(stats[0]) == int(want_levels.max()) + 1, f"{what}: depth {stats[0]}"
    assert int(stats[1]) == int(reached.sum()), f"{what}: reached {stats[1]}"
    assert int(stats[2]) == int(deg[reached].sum()), f"{what}: edges {stats[2]}"
    assert int(stats[3]) == bad_entries, f"{what}: malformed entries {stats[3]}"
    if parents is None:
        return
    assert parents[src] == src, f"{what}: parent of the source"
    assert np.all(parents[~reached] == -1), f"{what}: parent of an unreached vertex"
    v = np.flatnonzero(reached)
    v = v[v != src]
    p = parents[v]
    assert np.all((p >= 0) & (p < nv)), f"{what}: parent out of range"
    assert np.array_equal(want_levels[p], want_levels[v] - 1), f"{what}: parent not one level up"
    # the edge p -> v exists (checked on a sample for large graphs)
    if v.shape[0] > 20_000:
        pick = np.random.default_rng(0).choice(v.shape[0], 20_000, replace=False)
        v, p = v[pick], p[pick]
    assert np.all(has_edge(row, col, p, v)), f"{what}: parent without an edge to the vertex"


def csr(src, dst, nv, symmetric=False):
    return w.csr_from_edges(np.asarray(src), np.asarray(dst), nv, symmetric=symmetric)


def test_single_vertex_and_isolated_source(gpu_lib):
    row, col = np.zeros(2, np.int64), np.zeros(0, np.int32)
    levels, parents, stats = run(gpu_lib, row, col, 0)
    check(row, col, 0, levels, parents, stats, "V=1")
    # a source with no edges in a larger graph
    s, d = w.uniform_random_edges(1000, 5000, seed=1)
    keep = (s != 7) & (d != 7)
    row, col = csr(s[keep], d[keep], 1000)
    levels, parents, stats = run(gpu_lib, row, col, 7)
    check(row, col, 7, levels, parents, stats, "isolated source")


def test_path_many_levels(gpu_lib):
    # a directed chain: one vertex per level, 3000 level barriers
    nv = 3000
    row, col = csr(np.arange(nv - 1), np.arange(1, nv), nv)
    log(f"[bfs] path V={nv}")
    levels, parents, stats = run(gpu_lib, row, col, 0)
    check(row, col, 0, levels, parents, stats, "path")
    levels, parents, stats = run(gpu_lib, row, col, 1500)
    check(row, col, 1500, levels, parents, stats, "path from the middle")


def test_star_overflows_the_stage(gpu_lib):
    # the hub's chunk discovers 200k vertices: more than LDS keeps, so they
    # are placed by the second walk over the edges
    nv = 200_001
    leaves = np.arange(1, nv)
    row, col = csr(np.zeros(nv - 1, np.int64), leaves, nv, symmetric=True)
    for src in (0, 12_345):
        levels, parents, stats = run(gpu_lib, row, col, src)
        check(row, col, src, levels, parents, stats, f"star from {src}")


def test_dense_multi_edges_and_self_loops(gpu_lib):
    nv = 300
    u, v = np.meshgrid(np.arange(nv), np.arange(nv), indexing="ij")
    s = np.concatenate([u.ravel(), np.arange(nv), u.ravel()[::7]])     # complete + self loops + repeats
    d = np.concatenate([v.ravel(), np.arange(nv), v.ravel()[::7]])
    row, col = csr(s, d, nv)
    levels, parents, stats = run(gpu_lib, row, col, 5)
    check(row, col, 5, levels, parents, stats, "dense")


def test_grid_long_diameter(gpu_lib):
    n = 300
    idx = np.arange(n * n).reshape(n, n)
    s = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    d = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    row, col = csr(s, d, n * n, symmetric=True)
    log(f"[bfs] grid {n}x{n}")
    levels, parents, stats = run(gpu_lib, row, col, int(idx[n // 2, n // 3]))
    check(row, col, int(idx[n // 2, n // 3]), levels, parents, stats, "grid")


@pytest.mark.parametrize("scale", [10, 14, 17])
def test_rmat(gpu_lib, scale):
    s, d = w.rmat_edges(scale, 16, w.seed_for(9, scale))
    nv = 1 << scale
    row, col = csr(s, d, nv, symmetric=True)
    deg = np.diff(row)
    g = np.random.default_rng(scale)
    sources = [int(np.argmax(deg)), int(g.choice(np.flatnonzero(deg > 0))), int(g.choice(np.flatnonzero(deg > 0)))]
    if np.any(deg == 0):
        sources.append(int(np.flatnonzero(deg == 0)[0]))
    for src in sources:
        levels, parents, stats = run(gpu_lib, row, col, src)
        check(row, col, src, levels, parents, stats, f"rmat scale {scale} from {src}")
    log(f"[bfs] rmat scale {scale} ok")


def test_directed_with_unreachable_parts(gpu_lib):
    nv = 50_000
    s, d = w.uniform_random_edges(nv, 120_000, seed=3)
    row, col = csr(s, d, nv)
    for src in (0, 1, 49_999):
        levels, parents, stats = run(gpu_lib, row, col, src)
        check(row, col, src, levels, parents, stats, f"directed from {src}")


def test_without_parents(gpu_lib):
    s, d = w.rmat_edges(12, 8, w.seed_for(9, 1))
    row, col = csr(s, d, 1 << 12, symmetric=True)
    src = int(np.argmax(np.diff(row)))
    levels, parents, stats = run(gpu_lib, row, col, src, with_parents=False)
    assert parents is None
    check(row, col, src, levels, None, stats, "no parents")


def test_malformed_entries_are_skipped(gpu_lib):
    # columns outside [0, V) and a row range past E are skipped and counted
    nv = 1000
    s, d = w.uniform_random_edges(nv, 8000, seed=5)
    s[:50] = nv - 1          # the last vertex has out-edges (which its bad range hides)
    row, col = csr(s, d, nv)
    bad_col = col.copy()
    g = np.random.default_rng(6)
    pos = g.choice(int(row[nv - 1]), 40, replace=False)   # not in the last vertex's row
    bad_col[pos[:20]] = nv + 5
    bad_col[pos[20:]] = -3
    bad_row = row.copy()
    bad_row[nv] = row[nv] + 10  # the last vertex's range ends past E
    levels, parents, stats = run(gpu_lib, bad_row, bad_col, 0)
    # expected: the same graph without those entries and without the last
    # vertex's out-edges
    src_of = np.repeat(np.arange(nv), np.diff(row))
    ok = np.ones(col.shape[0], bool)
    ok[pos] = False
    ok[src_of == nv - 1] = False
    row2, col2 = csr(src_of[ok], col[ok], nv)
    want = oracle.bfs_levels(row2, col2, 0)
    assert np.array_equal(levels, want)
    reached = want >= 0
    assert reached[nv - 1], "the test wants the last vertex reached"
    # malformed entries are met (and counted) only in rows of reached vertices
    bad_cols_met = int(np.sum(np.isin(np.arange(col.shape[0]), pos) & reached[src_of]))
    assert int(stats[3]) == bad_cols_met + 1
    deg = np.diff(row)
    deg[nv - 1] = 0
    assert int(stats[2]) == int(deg[reached].sum())
    # parents stay valid in the graph without the malformed entries
    stats2 = np.array([stats[0], stats[1], np.diff(row2)[reached].sum(), 0])
    check(row2, col2, 0, levels, parents, stats2, "malformed")


def test_decreasing_row_offsets_are_refused(gpu_lib):
    nv = 500
    s, d = w.uniform_random_edges(nv, 3000, seed=8)
    row, col = csr(s, d, nv)
    bad_row = row.copy()
    bad_row[100] = bad_row[102] + 1   # row[99] <= row[100] > row[101]: one decreasing step
    bad_row[300] = -1                 # row[299] > row[300]: another
    levels, parents, stats = run(gpu_lib, bad_row, col, 0)
    assert np.all(levels == -1) and np.all(parents == -1)
    assert stats.tolist() == [0, 0, 0, 2]


@pytest.mark.parametrize("groups", [1, 2, 8])
def test_groups_per_cu(gpu_lib, groups):
    s, d = w.rmat_edges(15, 16, w.seed_for(9, 2))
    row, col = csr(s, d, 1 << 15, symmetric=True)
    src = int(np.argmax(np.diff(row)))
    levels, parents, stats = run(gpu_lib, row, col, src, params=gpu_lib.Params(0, 0, groups, 0))
    check(row, col, src, levels, parents, stats, f"groups {groups}")
    assert gpu_lib.lscan_last_launch().groups_per_cu <= groups


def test_repeated_calls_regrowth_and_two_streams(gpu_lib):
    graphs = []
    for k, scale in enumerate((9, 13, 11, 15)):
        s, d = w.rmat_edges(scale, 8, w.seed_for(9, 20 + k))
        row, col = csr(s, d, 1 << scale, symmetric=True)
        graphs.append((row, col, int(np.argmax(np.diff(row)))))
    for rep in range(3):
        for row, col, src in graphs:  # the workspace grows, tags keep advancing
            levels, parents, stats = run(gpu_lib, row, col, src)
            check(row, col, src, levels, parents, stats, f"repeat {rep} V={row.shape[0] - 1}")
    # alternate two streams without synchronising in between
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for k in range(4):
        row, col, src = graphs[k % len(graphs)]
        st = s1 if k % 2 == 0 else s2
        with torch.cuda.stream(st):
            rd, cd = dev(row, np.int64), dev(col, np.int32)
            outs.append((row, col, src, gpu_lib.bfs(rd, cd, src, stream=st), (rd, cd)))
    torch.cuda.synchronize()
    for row, col, src, (lv, pa, stt), _ in outs:
        check(row, col, src, lv.cpu().numpy(), pa.cpu().numpy(), stt.cpu().numpy(), "two streams")


def test_tag_range_reset(gpu_lib):
    # each call takes V + 3 tags; at 2^26 vertices the 32-bit tag space runs
    # out after 63 calls and the flag words are cleared: every result stays right
    nv = 1 << 26
    row = torch.zeros(nv + 1, dtype=torch.int64, device="cuda")
    row[-1] = 2       # vertex nv - 1 has two edges: to 3 and to itself
    col = torch.tensor([3, nv - 1], dtype=torch.int32, device="cuda")
    log("[bfs] tag reset, V=2^26, 70 calls")
    levels = torch.empty(nv, dtype=torch.int32, device="cuda")
    for k in range(70):
        src = nv - 1 if k % 2 else 3
        lv, _, stats = gpu_lib.bfs(row, col, src, levels=levels, parents=False)
        gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
        s = stats.cpu().numpy()
        if src == 3:
            assert s.tolist() == [1, 1, 0, 0], (k, s)
            assert int(lv[3].item()) == 0 and int((lv >= 0).sum().item()) == 1
        else:
            assert s.tolist() == [2, 2, 2, 0], (k, s)   # levels 0, 1; itself and vertex 3; its two edges
            assert int(lv[3].item()) == 1 and int(lv[nv - 1].item()) == 0
            assert int((lv >= 0).sum().item()) == 2
    del row, levels
    torch.cuda.empty_cache()


def test_empty_graph(gpu_lib):
    stats = torch.full((4,), 9, dtype=torch.int64, device="cuda")
    row = torch.zeros(1, dtype=torch.int64, device="cuda")
    col = torch.zeros(0, dtype=torch.int32, device="cuda")
    _, _, stats = gpu_lib.bfs(row, col, 0, stats=stats)
    torch.cuda.synchronize()
    assert stats.cpu().tolist() == [0, 0, 0, 0]


def test_full_size_rmat_scale22(gpu_lib):
    # the measured configuration: R-MAT, 2^22 vertices, edge factor 16,
    # both directions (134M column entries)
    row, col = w.rmat_csr_torch(22, 16, w.seed_for(9), device="cuda")
    log(f"[bfs] full size: V=2^22, E={col.shape[0]}")
    rh, ch = row.cpu().numpy(), col.cpu().numpy()
    deg = np.diff(rh)
    src = int(np.argmax(deg))
    levels, parents, stats = gpu_lib.bfs(row, col, src)
    gpu_lib.lscan_check(torch.cuda.current_stream().cuda_stream)
    check(rh, ch, src, levels.cpu().numpy(), parents.cpu().numpy(), stats.cpu().numpy(), "rmat scale 22")
    del row, col, levels, parents
    torch.cuda.empty_cache()
