"""Performance model of the Strassen-fused kernels on MI355X.

The Analysis section of the paper models one kernel as
    T = max(T_flop, T_smop, T_gmop)
with per-thread-block counts of arithmetic, shared-memory and global-memory
operations (eqs. n_flop, AB_gr_rs, AB_sr, C_rg) divided by the corresponding
device throughputs, after choosing the blocking that keeps each ratio below
the machine balance (eqs. constrain_glb, constrain_sha_bdw).  The same form
is used here with the gfx950 resources the kernels actually use:

  flop   MFMA flops                    / (CUs * MFMA flop/clk/CU * clock)
  lds    LDS bytes written + read      / (CUs * 128 B/clk * clock)
  l2     L2 -> CU operand bytes        / (CUs * L2 B/clk/CU * clock)
  hbm    algorithmic HBM bytes         / HBM bandwidth

per launch (one race-free batch of products of one variant), with the
counts of one workgroup tile:
  operand bytes per k-tile   (W_A * MT + W_B * NT) * KT * b_in        (l2)
  LDS bytes per k-tile       (MT + NT) * KT * b_lds * planes           (stores)
                             + waves * (WM + WN) * KT * b_lds * planes (fragment reads)
  C bytes per tile           2 * 4 * W_C * MT * NT                     (epilogue)
and a wave-quantisation factor ceil(W / S) / (W / S) for W workgroups on S
slots (the paper's inter-kernel parallelism argument for small problems).
A launch costs the maximum of its resource times, times that factor, plus a
fixed launch overhead.  The constants below are public MI355X figures, the
L2 and LDS widths are per-CU figures of the CDNA generation, and the clock
is the one measured under the fp32 GEMM (GRBM_GUI_ACTIVE).
"""
import math

from . import _binding as B

CUS = 256
CLOCK_HZ = 2.31e9            # measured under load (nominal 2.4 GHz)
MFMA_FLOP_PER_CLK_CU = {"f32": 256.0, "16bit": 4096.0}
LDS_B_PER_CLK_CU = 128.0
L2_B_PER_CLK_CU = 64.0
HBM_B_PER_S = 8.0e12
LAUNCH_S = 6e-6

TILES = {  # (MT, NT, KT, waves, workgroups per CU)
    ("f32", False): (128, 128, 32, 4, 2),
    ("f32", True): (256, 256, 32, 8, 1),   # KT 16 above four operand terms
    ("16bit", False): (128, 128, 32, 4, 2),
    ("16bit", True): (256, 256, 32, 8, 1),
    ("x3", False): (128, 128, 32, 4, 2),
    ("x3", True): (256, 256, 16, 8, 1),
}


def _batches(levels):
    """[(W_A, W_B, W_C, products)] per launch, in launch order."""
    rc, ins = B.strassen_plan_instances(levels)
    if rc < 0:
        raise ValueError("bad levels")
    out = {}
    for p in ins:
        w = out.setdefault(p.launch, [p.n_a, p.n_b, p.n_c, 0])
        w[3] += 1
    return [tuple(out[i]) for i in sorted(out)]


def _use_large(sm, sn, batch):
    per = math.ceil(sm / 256) * math.ceil(sn / 256)
    return per >= 128 and per * batch >= 256


def predict(m, n, k, levels, kind="f32"):
    """Predicted seconds of one call; kind in {'f32', '16bit', 'x3'}.
    Returns (total_seconds, [per-launch dicts])."""
    dt = {"f32": B.STRASSEN_F32, "16bit": B.STRASSEN_BF16, "x3": B.STRASSEN_F32}[kind]
    mode = B.STRASSEN_MODE_BF16X3 if kind == "x3" else B.STRASSEN_MODE_PLAIN
    rc, info = B.strassen_plan_info(m, n, k, levels, dt, mode)
    if rc != 0:
        raise ValueError("plan_info failed (%d)" % rc)
    sm, sn, sk = info.sub_m, info.sub_n, info.sub_k
    b_in = 2 if kind == "16bit" else 4
    b_lds = 4 if kind == "f32" else 2
    planes = 2 if kind == "x3" else 1
    mfma_mult = 3 if kind == "x3" else 1
    rate_kind = "f32" if kind == "f32" else "16bit"
    launches = []
    total = 0.0
    for wa, wb, wc, batch in _batches(levels):
        large = _use_large(sm, sn, batch)
        mt, nt, kt, waves, slots_per_cu = TILES[(kind, large)]
        if kind == "f32" and large and wa + wb > 4:
            kt = 16
        tiles = math.ceil(sm / mt) * math.ceil(sn / nt) * batch
        ktiles = math.ceil(sk / kt)
        wm, wn = (mt // 2, nt // (waves // 2))
        flops = 2.0 * mt * nt * kt * ktiles * tiles * mfma_mult
        lds = ((mt + nt) * kt * b_lds * planes + waves * (wm + wn) * kt * b_lds * planes) * ktiles * tiles
        l2 = (wa * mt + wb * nt) * kt * b_in * ktiles * tiles
        hbm = batch * (b_in * (wa * sm * sk + wb * sk * sn) + 8 * wc * sm * sn)
        t = {
            "flop": flops / (CUS * MFMA_FLOP_PER_CLK_CU[rate_kind] * CLOCK_HZ),
            "lds": lds / (CUS * LDS_B_PER_CLK_CU * CLOCK_HZ),
            "l2": l2 / (CUS * L2_B_PER_CLK_CU * CLOCK_HZ),
            "hbm": hbm / HBM_B_PER_S,
        }
        slots = CUS * slots_per_cu
        quant = math.ceil(tiles / slots) / (tiles / slots)
        bound = max(t, key=t.get)
        secs = t[bound] * quant + LAUNCH_S
        total += secs
        launches.append({"variant": (wa, wb, wc), "batch": batch, "tile": (mt, nt, kt),
                         "workgroups": tiles, "bound": bound, "seconds": secs,
                         "quantisation": quant, **{"t_" + r: v for r, v in t.items()}})
    return total, launches
