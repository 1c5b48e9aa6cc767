"""The performance model (Analysis section, T = max of the resource times per
launch, with the staging VALU work added to the MFMA time, plus wave
quantisation and launch overhead) against facts it must reproduce: the flop
term is the executed MFMA work of the plan, launches are the plan's race-free
batches, small problems lose to quantisation, one level pays for fp32 but not
for 16-bit operands, and the 16-bit two-level path leaves the MFMA bound.
Host only: plan queries need no GPU."""
import math

import pytest

import paper_1808_07984_amd as sg
from paper_1808_07984_amd import model


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_launches_are_the_plans_batches(levels):
    rc, info = sg.strassen_plan_info(4096, 4096, 4096, levels)
    assert rc == 0
    _, launches = model.predict(4096, 4096, 4096, levels)
    assert len(launches) == info.n_launches == [1, 4, 16][levels]
    assert sum(l["batch"] for l in launches) == 7 ** levels


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_flop_term_is_executed_mfma_work(levels):
    """Full tiles at 16384: sum over launches of t_flop x MFMA rate equals the
    plan's executed flops 7^L * 2 * s^3."""
    n = 16384
    _, info = sg.strassen_plan_info(n, n, n, levels)
    _, launches = model.predict(n, n, n, levels)
    rate = model.CUS * model.MFMA_FLOP_PER_CLK_CU["f32"] * model.CLOCK_HZ
    flops = sum(l["t_flop"] for l in launches) * rate
    assert math.isclose(flops, info.executed_flops, rel_tol=1e-12)
    assert all(l["bound"] == "flop" for l in launches)


def test_plain_gemm_time_is_flops_over_peak_plus_staging():
    """Full tiles: flops over the MFMA peak, plus one VALU op per staged
    element (the sign multiply), 512 elements per 256x256 tile and k step."""
    n = 16384
    t, (l,) = model.predict(n, n, n, 0)
    ideal = 2.0 * n ** 3 / (model.CUS * model.MFMA_FLOP_PER_CLK_CU["f32"] * model.CLOCK_HZ)
    staging = (256 + 256) * n * (n // 256) ** 2 / (model.CUS * model.VALU_OPS_PER_CLK_CU * model.CLOCK_HZ)
    assert l["quantisation"] == 1.0
    assert math.isclose(l["t_flop"], ideal, rel_tol=1e-12)
    assert math.isclose(l["t_valu"], staging, rel_tol=1e-12)
    assert math.isclose(t, ideal + staging + model.LAUNCH_S, rel_tol=1e-12)


def test_strassen_pays_at_large_sizes_only():
    """fp32: one level predicted faster than plain at 16384, slower at 1024
    (fewer, emptier launches: wave quantisation and launch overhead)."""
    big0, _ = model.predict(16384, 16384, 16384, 0)
    big1, _ = model.predict(16384, 16384, 16384, 1)
    small0, _ = model.predict(1024, 1024, 1024, 0)
    small1, ls = model.predict(1024, 1024, 1024, 1)
    assert big1 < big0
    assert small1 > small0
    assert any(l["quantisation"] > 1.0 for l in ls)


def test_16bit_two_level_leaves_the_mfma_bound():
    """At 16384 the 16-bit two-level launches are bound by their four-term
    operand sums (VALU), HBM or L2->CU operand traffic, not by the MFMAs,
    while fp32 stays MFMA bound at every level."""
    _, ls = model.predict(16384, 16384, 16384, 2, "16bit")
    assert all(l["bound"] in ("valu", "hbm", "l2") for l in ls)
    for L in (0, 1, 2):
        _, lf = model.predict(16384, 16384, 16384, L, "f32")
        assert all(l["bound"] == "flop" for l in lf)
    _, l0 = model.predict(16384, 16384, 16384, 0, "16bit")
    assert l0[0]["bound"] in ("flop", "lds")


def test_16bit_one_level_costs_more_than_it_saves():
    """16-bit MFMAs are so fast that forming two-term operand sums (a convert
    and an FMA per element) costs more than the eighth of the flops one level
    saves: plain is predicted faster at 16384, as measured (8.4 ms plain, 12.2
    ms one level, bf16)."""
    n = 16384
    t0, _ = model.predict(n, n, n, 0, "16bit")
    t1, ls = model.predict(n, n, n, 1, "16bit")
    assert t1 > t0
    assert any(l["t_valu"] > 0.5 * l["t_flop"] for l in ls)
    f0, _ = model.predict(n, n, n, 0, "f32")
    f1, _ = model.predict(n, n, n, 1, "f32")
    assert f1 < f0


def test_compensated_mode_triples_the_flop_term():
    n = 8192
    _, f = model.predict(n, n, n, 0, "16bit")
    _, x = model.predict(n, n, n, 0, "x3")
    assert math.isclose(x[0]["t_flop"], 3 * f[0]["t_flop"], rel_tol=1e-12)


# Automatic tile choice: the library picks, per launch, the tile whose waves
# of workgroups cost less; the model mirrors that rule.  plan_info reports the
# tile of the launch with the most operand terms.
@pytest.mark.parametrize("m,n,k", [(16384, 16384, 16384), (12288, 12288, 12288), (10240, 10240, 10240),
                                   (8192, 8192, 8192), (6144, 6144, 6144), (4096, 4096, 4096),
                                   (16384, 16384, 1024), (15001, 17003, 9007), (3000, 20000, 5000),
                                   (1024, 1024, 1024)])
@pytest.mark.parametrize("levels", [0, 1, 2])
def test_tile_choice_matches_model(m, n, k, levels):
    info = sg.plan_info(m, n, k, levels)
    rc, ins = sg.strassen_plan_instances(levels)
    assert rc >= 0
    launches = {}
    for p in ins:
        w = launches.setdefault(p.launch, [p.n_a + p.n_b, 0])
        w[1] += 1
    terms, batch = max(launches.values(), key=lambda v: v[0])
    widest = [b for t, b in launches.values() if t == terms][0]
    large = model._use_large(info.sub_m, info.sub_n, info.sub_k, widest, True)
    assert info.tile_m == (256 if large else 128)


@pytest.mark.parametrize("m,levels,tile", [(16384, 0, 256), (16384, 1, 256), (12288, 0, 256),
                                           (10240, 0, 128), (6144, 0, 128), (6144, 2, 128),
                                           (4096, 0, 256), (1024, 0, 128)])
def test_tile_choice_measured_cases(m, levels, tile):
    """Shapes where the faster tile was measured on MI355X (fp32): full 256x256
    waves keep 256x256; 4.5-wave or 2.25-wave launches take 128x128."""
    assert sg.plan_info(m, m, m, levels).tile_m == tile
