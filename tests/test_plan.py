"""Host planner of the HIP library, through the C ABI (no GPU needed).

Pins: the products the library launches satisfy the bilinear (Brent)
identities of block matrix multiplication on the 2x2 and 4x4 partitions; the
one-level products are exactly the seven of the Method section, eq.
gpu_allops; the variant multiset equals table tab:perfeq_level2; every launch
is race free (pairwise disjoint C write sets, one variant); beta is applied by
exactly one, the first, update of every C block.
"""
import itertools
from collections import Counter

import numpy as np
import pytest

import paper_1808_07984_amd as sg
from conftest import parse_scheme, read_golden


def _instances(levels):
    rc, ins = sg.strassen_plan_instances(levels)
    assert rc == 7 ** levels
    return ins


def _terms(blocks, signs, n):
    return sorted((int(blocks[t]), int(signs[t])) for t in range(n))


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_brent_identities(levels):
    """sum_p U_p[a] V_p[b] W_p[c] equals the block matrix-multiplication
    tensor: 1 iff a = (i, l), b = (l, j), c = (i, j)."""
    d = 2 ** levels
    nb = d * d
    T = np.zeros((nb, nb, nb), dtype=np.int64)
    for p in _instances(levels):
        u = np.zeros(nb, dtype=np.int64)
        v = np.zeros(nb, dtype=np.int64)
        w = np.zeros(nb, dtype=np.int64)
        for t in range(p.n_a):
            u[p.a_block[t]] += p.a_sign[t]
        for t in range(p.n_b):
            v[p.b_block[t]] += p.b_sign[t]
        for t in range(p.n_c):
            w[p.c_block[t]] += p.c_sign[t]
        T += np.einsum("a,b,c->abc", u, v, w)
    want = np.zeros_like(T)
    for i, l, j in itertools.product(range(d), repeat=3):
        want[i * d + l, l * d + j, i * d + j] = 1
    assert np.array_equal(T, want)


def test_one_level_matches_paper_scheme():
    paper = sorted((_terms([q for q, _ in a], [s for _, s in a], len(a)),
                    _terms([q for q, _ in b], [s for _, s in b], len(b)),
                    _terms([q for q, _ in c], [s for _, s in c], len(c)))
                   for _, a, b, c in parse_scheme())
    ours = sorted((_terms(p.a_block, p.a_sign, p.n_a), _terms(p.b_block, p.b_sign, p.n_b),
                   _terms(p.c_block, p.c_sign, p.n_c)) for p in _instances(1))
    assert ours == paper


def test_variant_counts_match_paper_table():
    want = {}
    for ln in read_golden("variant_counts.txt"):
        lv, _, wa, wb, wc, cnt = ln.split()
        want.setdefault(int(lv), Counter())[(int(wa), int(wb), int(wc))] = int(cnt)
    for lv in (0, 1, 2):
        got = Counter((p.n_a, p.n_b, p.n_c) for p in _instances(lv))
        assert got == want[lv], lv


def test_paper_streaming_stages_are_race_free_in_our_table():
    """The stage table (tab:gpu_streaming) runs products of one stage on two
    streams concurrently; with our one-level products, products of a stage on
    different streams write disjoint C quadrants."""
    ins = _instances(1)
    paper = parse_scheme()

    def cset(prod_idx):
        _, a, b, c = paper[prod_idx]
        key = (_terms([q for q, _ in a], [s for _, s in a], len(a)),
               _terms([q for q, _ in b], [s for _, s in b], len(b)))
        for p in ins:
            if (_terms(p.a_block, p.a_sign, p.n_a), _terms(p.b_block, p.b_sign, p.n_b)) == key:
                return {p.c_block[t] for t in range(p.n_c)}
        raise AssertionError("product %d not found" % prod_idx)

    stages = {}
    for ln in read_golden("streaming_stages.txt"):
        st, prod, stream = map(int, ln.split())
        stages.setdefault(st, {}).setdefault(stream, []).append(prod)
    for st, streams in stages.items():
        if len(streams) < 2:
            continue
        s0 = set().union(*[cset(p) for p in streams[0]])
        s1 = set().union(*[cset(p) for p in streams[1]])
        assert not (s0 & s1), st


@pytest.mark.parametrize("levels,launches", [(0, 1), (1, 4), (2, 16)])
def test_batches_race_free_and_complete(levels, launches):
    ins = _instances(levels)
    by_launch = {}
    for p in ins:
        by_launch.setdefault(p.launch, []).append(p)
    assert sorted(by_launch) == list(range(launches))
    # launch order is non-decreasing in the returned list
    assert [p.launch for p in ins] == sorted(p.launch for p in ins)
    for lid, ps in by_launch.items():
        assert len({(p.n_a, p.n_b, p.n_c) for p in ps}) == 1, lid
        assert len(ps) <= 8
        blocks = [p.c_block[t] for p in ps for t in range(p.n_c)]
        assert len(blocks) == len(set(blocks)), lid
    # every product appears once
    keys = [(tuple(_terms(p.a_block, p.a_sign, p.n_a)), tuple(_terms(p.b_block, p.b_sign, p.n_b)))
            for p in ins]
    assert len(set(keys)) == len(keys) == 7 ** levels
    # a lower bound on launches: writers of the most-written C block
    writers = Counter(p.c_block[t] for p in ins for t in range(p.n_c))
    assert launches == max(writers.values())


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_beta_applied_once_by_first_update(levels):
    seen = {}
    for p in _instances(levels):
        for t in range(p.n_c):
            blk = p.c_block[t]
            if blk not in seen:
                assert p.c_first[t] == 1
                seen[blk] = p.launch
            else:
                assert p.c_first[t] == 0
    assert len(seen) == 4 ** levels


@pytest.mark.parametrize("m,n,k,levels", [
    (16384, 16384, 16384, 1), (16384, 16384, 16384, 2), (15001, 17003, 9007, 2),
    (3000, 20000, 5000, 2), (1024, 1024, 1024, 1), (1, 1, 1, 2), (3, 5, 7, 2), (16384, 16384, 512, 2)])
def test_plan_geometry(m, n, k, levels):
    info = sg.plan_info(m, n, k, levels)
    d = 2 ** levels
    assert info.blocks_per_dim == d
    assert info.sub_m == -(-m // d)
    # n and k extents are rounded up to the 4-element vector width at levels >= 1
    for got, dim in ((info.sub_n, n), (info.sub_k, k)):
        base = -(-dim // d)
        want = base if levels == 0 else -(-base // 4) * 4
        assert got == want
        assert d * got >= dim
    assert info.n_instances == 7 ** levels
    assert info.executed_flops == 7 ** levels * 2.0 * info.sub_m * info.sub_n * info.sub_k
    assert info.classical_flops == 2.0 * m * n * k


def test_executed_flop_ratio_on_divisible_sizes():
    """7/8 and 49/64 of the classical flops (Method section; ideal 1.3x at two
    levels, Experiment section)."""
    for L, ratio in ((1, 7 / 8), (2, 49 / 64)):
        info = sg.plan_info(16384, 16384, 16384, L)
        assert info.executed_flops / info.classical_flops == pytest.approx(ratio, rel=0, abs=0)
