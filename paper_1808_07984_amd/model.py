"""Performance model of the Strassen-fused kernels on MI355X.

The Analysis section of the paper models one kernel as
    T = max(T_flop, T_smop, T_gmop)
with per-thread-block counts of arithmetic, shared-memory and global-memory
operations (eqs. n_flop, AB_gr_rs, AB_sr, C_rg) divided by the corresponding
device throughputs, after choosing the blocking that keeps each ratio below
the machine balance (eqs. constrain_glb, constrain_sha_bdw).  The same form
is used here with the gfx950 resources the kernels actually use:

  flop   MFMA flops                    / (CUs * MFMA flop/clk/CU * clock)
  valu   operand-staging VALU ops      / (CUs * 64 lane-ops/clk * clock)
  lds    LDS bytes written / (CUs * 128 B/clk * clock)
         + LDS bytes read  / (CUs * 256 B/clk * clock)
  l2     L2 -> CU operand bytes        / (CUs * L2 B/clk/CU * clock)
  hbm    algorithmic HBM bytes         / HBM bandwidth

per launch (one race-free batch of products of one variant), with the
counts of one workgroup tile.  The staging VALU work is added to the MFMA
time rather than overlapped with it: each wave issues its sums in order with
its MFMAs and meets a barrier every k-tile, and measured kernels lose about
the VALU/MFMA ratio (fp32 W > 1 kernels a few per cent; 16-bit one-level
launches more than the flops they save):
  operand bytes per k-tile   (W_A * MT + W_B * NT) * KT * b_in        (l2)
  LDS bytes per k-tile       (MT + NT) * KT * b_lds * planes           (stores)
                             + waves * (WM + WN) * KT * b_lds * planes (fragment reads)
  C bytes per tile           2 * 4 * W_C * MT * NT                     (epilogue)
  staging ops per k-tile     per element of each operand tile: fp32 one
                             multiply-add per term; 16-bit one pass-through
                             (single term) or a convert and an FMA per term
                             plus half a packed rounding; bf16x3 adds the
                             hi/lo split
and a wave-quantisation factor ceil(W / S) / (W / S) for W workgroups on S
slots (the paper's inter-kernel parallelism argument for small problems).
A launch costs max(T_flop + T_valu, T_lds, T_l2, T_hbm) times that factor,
plus a fixed launch overhead.  The constants below are public MI355X figures
or measured on it: the LDS widths with a microbenchmark (16-byte reads 256
B/clk/CU, 16-byte writes 125), the clock under the fp32 GEMM
(GRBM_GUI_ACTIVE), and the clock under sustained 16-bit MFMA work on random
operands, which is power limited (a pure 32x32x16 MFMA loop sustains
1.69-1.75 PFLOP/s, every instruction still 32 cycles: ~1.65 GHz).  16-bit
and compensated launches use that clock for every term.  The model leaves
out load latency and barrier waits, which it therefore underestimates for
the 16-bit kernels (see the measured MFMA-busy fractions).
"""
import math

from . import _binding as B

CUS = 256
CLOCK_HZ = 2.38e9            # measured under the fp32 GEMM (GRBM_GUI_ACTIVE per XCD)
CLOCK_16BIT_HZ = 1.65e9      # power-limited clock under 16-bit MFMA work, random operands
MFMA_FLOP_PER_CLK_CU = {"f32": 256.0, "16bit": 4096.0}
LDS_WRITE_B_PER_CLK_CU = 128.0
LDS_READ_B_PER_CLK_CU = 256.0
VALU_OPS_PER_CLK_CU = 64.0   # 4 SIMDs x 16 lanes
L2_B_PER_CLK_CU = 64.0
HBM_B_PER_S = 8.0e12
LAUNCH_S = 6e-6

TILES = {  # (MT, NT, KT, waves, workgroups per CU)
    ("f32", False): (128, 128, 32, 4, 2),
    ("f32", True): (256, 256, 32, 8, 1),   # KT 16 above four operand terms but (4,1,4), (4,2,2)
    ("16bit", False): (128, 128, 32, 4, 2),
    ("16bit", True): (256, 256, 64, 8, 1),  # KT 32 above four operand terms and for (1,2,2)
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


def _use_large(sm, sn, sk, batch, f32):
    """The library's automatic tile choice (wave-cost comparison for fp32)."""
    per = math.ceil(sm / 256) * math.ceil(sn / 256)
    if not f32:
        return per >= 128 and per * batch >= 256
    t128 = math.ceil(sm / 128) * math.ceil(sn / 128) * batch
    cost256 = math.ceil(per * batch / 256) * (sk + 62.5)
    pair = 0.5 * (1.045 * sk + 16.5)
    full, rest = divmod(t128, 512)
    cost128 = full * pair + (0.0 if rest == 0 else 0.65 * pair if rest <= 256 else pair)
    return cost256 <= cost128


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
        large = _use_large(sm, sn, sk, batch, kind == "f32")
        mt, nt, kt, waves, slots_per_cu = TILES[(kind, large)]
        if kind == "f32" and large and wa + wb > 4 and (wa, wb, wc) not in ((4, 1, 4), (4, 2, 2)):
            kt = 16
        if kind == "16bit" and large and (wa + wb > 4 or (wa, wb) == (1, 2)):
            kt = 32
        if kind == "x3" and large and wa + wb == 2:
            kt = 32
        tiles = math.ceil(sm / mt) * math.ceil(sn / nt) * batch
        ktiles = math.ceil(sk / kt)
        wm, wn = (mt // 2, nt // (waves // 2))
        flops = 2.0 * mt * nt * kt * ktiles * tiles * mfma_mult
        lds_w = (mt + nt) * kt * b_lds * planes * ktiles * tiles
        lds_r = waves * (wm + wn) * kt * b_lds * planes * ktiles * tiles
        l2 = (wa * mt + wb * nt) * kt * b_in * ktiles * tiles

        def staging(w):  # VALU lane-ops per element of one operand tile
            if kind == "f32":
                return float(w)
            if kind == "x3":
                return 2.0 * w + 3.0
            return 0.125 if w == 1 else 2.0 * w + 0.5
        valu = (mt * staging(wa) + nt * staging(wb)) * kt * ktiles * tiles
        hbm = batch * (b_in * (wa * sm * sk + wb * sk * sn) + 8 * wc * sm * sn)
        clock = CLOCK_HZ if kind == "f32" else CLOCK_16BIT_HZ
        t = {
            "flop": flops / (CUS * MFMA_FLOP_PER_CLK_CU[rate_kind] * clock),
            "valu": valu / (CUS * VALU_OPS_PER_CLK_CU * clock),
            "lds": (lds_w / LDS_WRITE_B_PER_CLK_CU + lds_r / LDS_READ_B_PER_CLK_CU) / (CUS * clock),
            "l2": l2 / (CUS * L2_B_PER_CLK_CU * clock),
            "hbm": hbm / HBM_B_PER_S,
        }
        slots = CUS * slots_per_cu
        quant = math.ceil(tiles / slots) / (tiles / slots)
        limits = {"compute": t["flop"] + t["valu"], "lds": t["lds"], "l2": t["l2"], "hbm": t["hbm"]}
        bound = max(limits, key=limits.get)
        secs = limits[bound] * quant + LAUNCH_S
        if bound == "compute":
            bound = "flop" if t["flop"] >= t["valu"] else "valu"
        total += secs
        launches.append({"variant": (wa, wb, wc), "batch": batch, "tile": (mt, nt, kt),
                         "workgroups": tiles, "bound": bound, "seconds": secs,
                         "quantisation": quant, **{"t_" + r: v for r, v in t.items()}})
    return total, launches
