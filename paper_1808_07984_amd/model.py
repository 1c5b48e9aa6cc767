"""Performance model of the Strassen-fused kernels on MI355X.

The Analysis section of the paper models one kernel as
    T = max(T_flop, T_smop, T_gmop)
with per-thread-block counts of arithmetic, shared-memory and global-memory
operations (eqs. n_flop, AB_gr_rs, AB_sr, C_rg) divided by the corresponding
device throughputs.  The same form is kept here, per workgroup and per round
of workgroups, with the gfx950 resources the kernels use and throughputs
measured on MI355X:

* a launch of W workgroups on S = CUs x (workgroups per CU) slots runs in
  rounds of at most S workgroups; a round of w workgroups puts
  c = ceil(w / CUs) of them on each of min(w, CUs) CUs;
* one round costs
      max(c * (T_flop + T_valu), c * T_lds, w/a * T_fetch) + w/a * T_C + T_round
  per CU, where
      T_flop   MFMA flops of one workgroup / (MFMA flop/clk/CU * clock)
      T_valu   operand-staging lane-ops / (64 lane-ops/clk/CU * clock): each
               wave issues its sums in order with its MFMAs and meets a
               barrier every k-tile, so staging adds to the MFMA time
      T_lds    LDS bytes written / 128 B/clk + read / 256 B/clk
      T_fetch  A-operand bytes / R_A + B-operand bytes / R_B (the operand
               bytes one workgroup requests over its k loop, every term of
               every sum counted)
      T_C      C bytes of the epilogue (a read and a write of 4 bytes per
               element per output) / R_C: the epilogue follows the k loop,
               so it adds
      T_round  a fixed cost per round (pipeline fill at the start of a tile,
               drain at its end);
* a launch costs the sum of its rounds, at least its algorithmic HBM bytes
  over 8 TB/s, plus a launch overhead.

R_A, R_B, R_C, T_round and the 0.85 factor of the 128 x 128 tile's operand
rates are fitted to the event times of every launch of squares 1024-16384 at
levels 0/1/2 (fp32, bf16 and the compensated mode, fused and formed).
Launches that load their operands straight into LDS (the single-term
products on 256 x 256 tiles, 16-bit or pre-split compensated) have no
staging lane-ops of their own (16-bit) or DIRECT_VALU of the staged split's
(pre-split: 0.4, fitted to the same table); their operand rates are those of
the staged loads.  They are per-CU rates
of latency-bound loads, not bandwidths: the sixteen-bit kernels reach about
a third of their MFMA peak on the plain product, and their multi-term launches
are set by how many operand bytes a CU can keep in flight.  The B operand
(n-contiguous, staged through the paired layout) costs about twice the A
operand per byte.  That is not the tile walk's panel sharing (the 32
workgroups one XCD runs at once are 4 tile rows x 8 columns, so each A panel
is shared eight ways and each B panel four): walking groups of eight rows
instead, which reverses the sharing, left the B-heavy compensated launches
unchanged (-0.4 to -0.6 %, results identical).  Clocks are the
measured ones: fp32 under the GEMM (GRBM_GUI_ACTIVE), 16-bit under sustained
MFMA work on random operands, which is power limited (1.65-1.78 GHz in the
library's MFMA rate probe, strassen_probe_mfma).

Also modelled: the formed schedules' sum kernels (streaming, at a measured
5 TB/s) and the one-level schedule's chained launches (two products per
workgroup, one epilogue).
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
R_A_B_PER_S_CU = 58e9        # A-operand bytes per second per CU (fitted)
R_B_B_PER_S_CU = 29e9        # B-operand bytes per second per CU (fitted)
R_C_B_PER_S_CU = 26e9        # epilogue C bytes per second per CU (fitted)
SMALL_TILE_FETCH = 0.85      # 128x128 tile: operand time factor (fitted)
# operands loaded straight into LDS: factor on the staging lane-ops (none for
# 16-bit data; for pre-split compensated data, fitted: the units' hi and lo
# halves are still regrouped per fragment)
DIRECT_VALU = {"16bit": 0.0, "x3": 0.4}
ROUND_S = 7e-6               # fixed cost per round of workgroups (fitted)
FORM_B_PER_S = 5.0e12        # sum-forming kernels, bytes read + written (measured)
HBM_B_PER_S = 8.0e12
LAUNCH_S = 6e-6

OCCUPANCY = {False: 2, True: 1}   # workgroups per CU: 128x128 (4 waves), 256x256 (8 waves)


def tile(kind, large, wa, wb, wc, a_kc=True, b_kc=False):
    """(MT, NT, KT) the library instantiates for this variant.  kind in
    {'f32', '16bit', 'x3'}; a_kc / b_kc: A and B k-contiguous in memory
    (row-major A, row-major B: a_kc True, b_kc False)."""
    if not large:
        return 128, 128, 32
    if kind == "f32":
        split = a_kc and not b_kc and wa == 4 and (wb, wc) in ((1, 4), (2, 2))
        return 256, 256, 16 if wa + wb > 4 and not split else 32
    if kind == "16bit":
        return 256, 256, 64 if wa + wb <= 4 and (wa, wb) != (1, 2) else 32
    return 256, 256, 32 if wa + wb == 2 and a_kc and not b_kc else 16


def _staging(kind, w):
    """VALU lane-ops per element of one operand tile for a w-term sum: fp32
    one multiply-add per term; 16-bit one pass-through (single term) or a
    convert and an FMA per term plus half a packed rounding; the compensated
    mode adds the hi/lo split."""
    if kind == "f32":
        return float(w)
    if kind == "x3":
        return 2.0 * w + 3.0
    return 0.125 if w == 1 else 2.0 * w + 0.5


def direct_loads(kind, large, wa, wb, pre_b=True):
    """Whether the library loads this variant's in-bounds k-tiles straight
    into LDS: single-term products with A and B as stored on 256x256 tiles,
    16-bit operands or pre-split compensated ones (pre_b: B pre-split too,
    as in the formed schedules except for the one-level products that read B
    as stored)."""
    return large and wa == 1 and wb == 1 and (kind == "16bit" or (kind == "x3" and pre_b))


def launch(kind, large, wa, wb, wc, sm, sn, sk, batch, products_per_workgroup=1, direct=False):
    """Predicted seconds of one launch: `batch` products of sm x sk by
    sk x sn sub-blocks with W_A, W_B, W_C terms, each workgroup running
    `products_per_workgroup` products in turn (2 for a chained launch) and
    one epilogue of wc outputs; direct: the operands go straight into LDS
    (staging lane-ops scaled by DIRECT_VALU).  Returns a dict of the
    terms."""
    mt, nt, kt = tile(kind, large, wa, wb, wc)
    b_in = 2 if kind == "16bit" else 4
    b_lds = 4 if kind == "f32" else 2
    planes = 2 if kind == "x3" else 1
    mult = 3 if kind == "x3" else 1
    clock = CLOCK_HZ if kind == "f32" else CLOCK_16BIT_HZ
    rate = MFMA_FLOP_PER_CLK_CU["f32" if kind == "f32" else "16bit"]
    waves = 8 if large else 4
    wm, wn = mt // 2, nt // (waves // 2)
    ktiles = math.ceil(sk / kt) * products_per_workgroup
    per_wg = {
        "flop": 2.0 * mt * nt * kt * ktiles * mult / (rate * clock),
        "valu": (DIRECT_VALU.get(kind, 1.0) if direct else 1.0)
                * (mt * _staging(kind, wa) + nt * _staging(kind, wb)) * kt * ktiles / (VALU_OPS_PER_CLK_CU * clock),
        "lds": ((mt + nt) * kt * b_lds * planes / LDS_WRITE_B_PER_CLK_CU
                + waves * (wm + wn) * kt * b_lds * planes / LDS_READ_B_PER_CLK_CU) * ktiles / clock,
        "fetch": (wa * mt / R_A_B_PER_S_CU + wb * nt / R_B_B_PER_S_CU) * kt * b_in * ktiles
                 * (1.0 if large else SMALL_TILE_FETCH),
        "epilogue": 8.0 * wc * mt * nt / R_C_B_PER_S_CU,
    }
    tiles = math.ceil(sm / mt) * math.ceil(sn / nt) * batch
    slots = CUS * OCCUPANCY[large]
    full, rest = divmod(tiles, slots)
    rounds = [slots] * full + ([rest] if rest else [])
    t = 0.0
    busy = {"compute": 0.0, "lds": 0.0, "fetch": 0.0}
    for w in rounds:
        active = min(w, CUS)
        per_cu = w / active
        c = math.ceil(w / CUS)
        r = {"compute": c * (per_wg["flop"] + per_wg["valu"]), "lds": c * per_wg["lds"],
             "fetch": per_cu * per_wg["fetch"]}
        t += max(r.values()) + per_cu * per_wg["epilogue"] + ROUND_S
        for key in busy:
            busy[key] += r[key]
    hbm = batch * (b_in * (wa * sm * sk + wb * sk * sn) * products_per_workgroup
                   + 8 * wc * sm * sn) / HBM_B_PER_S
    bound = max(busy, key=busy.get)
    if bound == "compute":
        bound = "flop" if per_wg["flop"] >= per_wg["valu"] else "valu"
    if hbm > t:
        t, bound = hbm, "hbm"
    flops_total = 2.0 * mt * nt * kt * ktiles * mult * tiles
    return {"variant": (wa, wb, wc), "batch": batch, "tile": (mt, nt, kt), "workgroups": tiles,
            "rounds": len(rounds), "bound": bound, "seconds": t + LAUNCH_S,
            "t_flop": flops_total / (CUS * rate * clock),
            "t_valu": per_wg["valu"] * tiles / CUS,
            "t_fetch": per_wg["fetch"] * tiles / CUS,
            "t_epilogue": per_wg["epilogue"] * tiles / CUS,
            "t_hbm": hbm}


def form(kind, rows, cols, n_sources, n_sums):
    """Seconds of one sum-forming launch: n_sources source blocks read once,
    n_sums sums of rows x cols written, streaming."""
    es = 2 if kind == "16bit" else 4
    return es * rows * cols * (n_sources + n_sums) / FORM_B_PER_S + LAUNCH_S


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
    """Predicted seconds of one fused call; kind in {'f32', '16bit', 'x3'}.
    Returns (total_seconds, [per-launch dicts])."""
    dt = {"f32": B.STRASSEN_F32, "16bit": B.STRASSEN_BF16, "x3": B.STRASSEN_F32}[kind]
    mode = B.STRASSEN_MODE_BF16X3 if kind == "x3" else B.STRASSEN_MODE_PLAIN
    rc, info = B.strassen_plan_info(m, n, k, levels, dt, mode)
    if rc != 0:
        raise ValueError("plan_info failed (%d)" % rc)
    sm, sn, sk = info.sub_m, info.sub_n, info.sub_k
    launches = []
    for wa, wb, wc, batch in _batches(levels):
        large = _use_large(sm, sn, sk, batch, kind == "f32")
        launches.append(launch(kind, large, wa, wb, wc, sm, sn, sk, batch,
                               direct=kind == "16bit" and direct_loads(kind, large, wa, wb)))
    return sum(l["seconds"] for l in launches), launches


def predict_formed(m, n, k, levels, kind="f32"):
    """Predicted seconds of one formed call (strassen_gemm_formed_ex), its
    launches one after another: the sum-forming launches (one level: one per
    operand, four quadrants into five sums, seven of A in the compensated
    mode, whose single quadrants are stored pre-split too; two levels: per
    operand five
    launches of eight blocks into seven sums and two of four into five, or
    into seven with the two single blocks in the compensated mode),
    then the single-term products in the fused schedule's batches (the
    one-level 16-bit chains, which save a C update and a launch, are not
    modelled).  Returns (total_seconds, [per-launch dicts or seconds])."""
    dt = {"f32": B.STRASSEN_F32, "16bit": B.STRASSEN_BF16, "x3": B.STRASSEN_F32}[kind]
    mode = B.STRASSEN_MODE_BF16X3 if kind == "x3" else B.STRASSEN_MODE_PLAIN
    rc, info = B.strassen_plan_info(m, n, k, levels, dt, mode)
    if rc != 0:
        raise ValueError("plan_info failed (%d)" % rc)
    sm, sn, sk = info.sub_m, info.sub_n, info.sub_k
    if levels == 1:
        forms = [form(kind, sm, sk, 4, 7 if kind == "x3" else 5), form(kind, sk, sn, 4, 5)]
    else:
        forms = [form(kind, rows, cols, src, out) for rows, cols in ((sm, sk), (sk, sn))
                 for src, out in [(8, 7)] * 5 + [(4, 7 if kind == "x3" else 5)] * 2]
    launches = []
    for wa, wb, wc, batch in _batches(levels):
        large = _use_large(sm, sn, sk, batch, kind == "f32")
        # compensated one level: the batch whose B operands are single
        # quadrants reads them as stored (fp32, split while staged)
        pre_b = levels == 2 or wb > 1
        launches.append(launch(kind, large, 1, 1, wc, sm, sn, sk, batch,
                               direct=direct_loads(kind, large, 1, 1, pre_b)))
    return sum(forms) + sum(l["seconds"] for l in launches), forms + launches


def parse_kernel(name):
    """(kind, large, (W_A, W_B, W_C) or None, chains or 0, direct) from a
    launch record's kernel name; kind None for the sum-forming kernels.
    direct: the variant loads its operands straight into LDS (16-bit and
    pre-split compensated single-term products as stored, 256x256 tiles)."""
    if name.startswith("form_"):
        return None, False, None, 0, False
    kind = "f32" if name.startswith("strassen_f32") else "x3" if "bf16x3" in name else "16bit"
    large = "256x256" in name
    pre_b = "bf16x3p," in name
    args = name[name.rindex("<") + 1:name.rindex(">")].split(",")
    untransposed = "tA" not in args and "tB" not in args
    if args[0] == "chained":
        return kind, large, None, int(args[1]), direct_loads(kind, large, 1, 1, pre_b)
    w = tuple(int(v) for v in args[:3])
    return kind, large, w, 0, untransposed and direct_loads(kind, large, w[0], w[1], pre_b)


def predict_record(kernel, batch, workgroups, sm, sn, sk, kind_hint=None):
    """Predicted seconds of one recorded launch (kernel name, batch,
    workgroups as the library records them) on sub-blocks sm x sk x sn.
    Sum-forming launches: one level, one operand's four quadrants into five
    sums of sm x sk; two levels (form_terms), `workgroups` distinct blocks
    into `batch` sums (kind_hint gives their element type)."""
    kind, large, variant, chains, direct = parse_kernel(kernel)
    if kind is None:
        fk = "16bit" if "16-bit" in kernel else "x3"
        if kernel.startswith("form_terms"):
            return form(kind_hint or fk, sm, sk, workgroups, batch)
        return form(kind_hint or fk, sm, sk, 4, batch)
    if chains:
        return launch(kind, large, 1, 1, 2, sm, sn, sk, chains, products_per_workgroup=2, direct=direct)["seconds"]
    return launch(kind, large, *variant, sm, sn, sk, batch, direct=direct)["seconds"]
