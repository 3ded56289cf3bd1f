"""CPU checks of the host symbolic analysis of the block-sparse solver
(csrc/symbolic.hpp), compiled with g++ into a small driver:
* the minimum-degree order equals a direct Python restatement of the rule
  (eliminate a node of smallest current degree, ties to the smallest index,
  join its neighbours into a clique) on random graphs;
* the tile pattern contains every non-zero of the numerical Cholesky factor
  of a random SPD matrix with the graph's block pattern (brute force), and is
  closed under tile-level elimination;
* the block column counts equal the non-zero blocks of that numerical
  factor column by column, and on a complete graph the block flop count is
  the dense one, close to (n d)^3 / 3."""
import os
import subprocess

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "symbolic_driver.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sym") / "symbolic_driver")
    r = subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, SRC], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr)
    return exe


def run(exe, n, d, ts, pairs, post=False):
    inp = f"{n} {d} {ts} {len(pairs)}\n" + "".join(f"{a} {b}\n" for a, b in pairs)
    out = subprocess.run([exe] + (["post"] if post else []), input=inp, capture_output=True, text=True,
                         check=True).stdout.split("\n")
    vals = {line.split()[0]: line.split()[1:] for line in out if line.strip()}
    order = [int(x) for x in vals["order"]]
    col_ptr = [int(x) for x in vals["col_ptr"]]
    rows = [int(x) for x in vals["row_idx"]]
    cols = [rows[col_ptr[J]:col_ptr[J + 1]] for J in range(int(vals["P"][0]))]
    run.counts = [int(x) for x in vals["counts"]]
    run.block_flops = float(vals["block_flops"][0])
    return order, cols


def py_min_degree(n, pairs):
    adj = [set() for _ in range(n)]
    for a, b in pairs:
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    done, order = set(), []
    for _ in range(n):
        v = min((u for u in range(n) if u not in done), key=lambda u: (len(adj[u]), u))
        order.append(v)
        done.add(v)
        nb = adj[v]
        for u in nb:
            adj[u] |= nb
            adj[u].discard(u)
            adj[u].discard(v)
        adj[v] = set()
    return order


def random_pairs(rng, n, m):
    pairs = set()
    for k in range(n - 1):
        pairs.add((k, k + 1))
    while len(pairs) < m:
        a, b = sorted(rng.choice(n, 2, replace=False))
        pairs.add((int(a), int(b)))
    return sorted(pairs)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_min_degree_matches_restatement(driver, seed):
    rng = np.random.default_rng(seed)
    n = 40
    pairs = random_pairs(rng, n, 70)
    order, _ = run(driver, n, 6, 16, pairs)
    assert sorted(order) == list(range(n))
    assert order == py_min_degree(n, pairs)


@pytest.mark.parametrize("ts,d,post", [(16, 6, False), (64, 6, False), (16, 3, False), (48, 6, True), (12, 3, True)])
def test_tile_pattern_covers_numeric_factor(driver, ts, d, post):
    rng = np.random.default_rng(ts + d)
    n = 30
    pairs = random_pairs(rng, n, 55)
    order, cols = run(driver, n, d, ts, pairs, post=post)
    pos = np.empty(n, int)
    pos[order] = np.arange(n)
    N = n * d
    H = np.zeros((N, N))
    for a in range(n):
        blk = rng.normal(size=(d, d))
        H[pos[a] * d:pos[a] * d + d, pos[a] * d:pos[a] * d + d] += blk @ blk.T + d * np.eye(d)
    for a, b in pairs:
        blk = 0.3 * rng.normal(size=(d, d))
        ra, rb = pos[a] * d, pos[b] * d
        H[ra:ra + d, rb:rb + d] += blk
        H[rb:rb + d, ra:ra + d] += blk.T
    H += 5 * N * np.eye(N) * 0 + np.eye(N) * np.abs(H).sum(1).max()   # diagonally dominant
    L = np.linalg.cholesky(H)
    P = len(cols)
    pattern = {(I, J) for J in range(P) for I in cols[J]}
    nz = np.argwhere(np.abs(L) > 1e-13)
    for r, c in nz:
        assert (r // ts, c // ts) in pattern
    for J in range(P):
        assert cols[J][0] == J and cols[J] == sorted(set(cols[J]))
        below = cols[J][1:]
        if below:
            parent = below[0]
            assert set(below[1:]) <= set(cols[parent])


def test_lattice_fill_is_moderate(driver):
    """The 10^3 lattice with 10% long-range edges and 48-wide tiles: the
    elimination-tree postorder keeps the tile fill well below the dense lower
    triangle (and below the plain minimum-degree order)."""
    p = synth.lattice_se3(batch=1, side=10)
    pairs = [tuple(x) for x in p["edge_ij"].tolist()]
    _, cols_md = run(driver, 1000, 6, 48, pairs)
    _, cols_po = run(driver, 1000, 6, 48, pairs, post=True)
    P = len(cols_po)
    n_md, n_po = sum(len(c) for c in cols_md), sum(len(c) for c in cols_po)
    assert n_po < n_md
    assert n_po < 0.5 * P * (P + 1) / 2


@pytest.mark.parametrize("seed,post", [(3, False), (4, True)])
def test_block_counts_equal_numeric_factor(driver, seed, post):
    rng = np.random.default_rng(seed)
    n, d = 36, 3
    pairs = random_pairs(rng, n, 60)
    order, _ = run(driver, n, d, 12, pairs, post=post)
    counts = run.counts
    pos = np.empty(n, int)
    pos[order] = np.arange(n)
    N = n * d
    H = np.zeros((N, N))
    for a, b in pairs:
        blk = rng.normal(size=(d, d))
        ra, rb = pos[a] * d, pos[b] * d
        H[ra:ra + d, rb:rb + d] += blk
        H[rb:rb + d, ra:ra + d] += blk.T
    H += np.eye(N) * (np.abs(H).sum(1).max() + 1.0)
    L = np.linalg.cholesky(H)
    for j in range(n):
        below = L[(j + 1) * d:, j * d:(j + 1) * d].reshape(n - j - 1, d, d)
        nzb = int(np.sum(np.abs(below).max(axis=(1, 2)) > 1e-13))
        assert counts[j] == nzb, (j, counts[j], nzb)


def test_block_flops_of_complete_graph(driver):
    n, d = 12, 6
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    run(driver, n, d, 12, pairs)
    assert run.counts == list(range(n - 1, -1, -1))
    # sum_j d^3/3 + m d^3 + m(m+1) d^3 with m = n-1-j
    m = np.arange(n)
    expect = float(np.sum(d ** 3 / 3 + m * d ** 3 + m * (m + 1) * d ** 3))
    assert abs(run.block_flops - expect) < 1e-9 * expect
    N = n * d
    assert abs(run.block_flops - N ** 3 / 3) < 0.2 * N ** 3 / 3
