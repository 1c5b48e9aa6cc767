"""Helpers shared by the GPU parity tests: input construction on the CPU,
device copies, and the tolerance of floating-point results.

Tolerance (reading of the paper, which states none): with
    scale = k * |alpha| * max|A| * max|B| + |beta| * max|C_in|
a result passes iff  max_ij |C_gpu - C*| <= tau_L * eps * scale,
    tau_L = 2^(L+1)  (2, 4, 8 for 0, 1, 2 levels),
    eps   = unit roundoff of the format the matrix cores consume
            (fp32 2^-23, bf16 2^-7, fp16 2^-10).  The compensated bf16x3
            mode is gated at 2^-16: its hi + lo split carries 16 significant
            bits, so each product is exact to about 2^-16 relative and the
            error grows like sqrt(k) 2^-16, about 128 / sqrt(k) in units of
            k 2^-23 (measured 5.6 at k = 520 on U[-1,1] data); the figure at
            2^-23 is reported beside it, not gated.  EPS["bf16x3"] below is
            that reporting unit.
k * eps * |A| |B| is the classical worst-case bound of a k-term fp32 dot
product (to first order); each Strassen level at most doubles the magnitude
of each operand sum and adds two roundings, so the factor 2 per level.
"""
import numpy as np
import torch

import oracle
from paper_1808_07984_amd import inputs

EPS = {"f32": 2.0 ** -23, "bf16": 2.0 ** -7, "f16": 2.0 ** -10, "bf16x3": 2.0 ** -23}
TORCH_DT = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16,
            "bf16x3": torch.float32}


def tau(levels):
    return 2.0 ** (levels + 1)


def e_norm(got, want, A, B, Cin, k, alpha, beta, eps):
    """max |got - want| in units of eps * (k |alpha| |A|max |B|max + |beta| |C|max)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    amax = float(np.abs(oracle._f64(A)).max()) if np.size(A) else 0.0
    bmax = float(np.abs(oracle._f64(B)).max()) if np.size(B) else 0.0
    cmax = float(np.nanmax(np.abs(oracle._f64(Cin)))) if (Cin is not None and beta != 0) else 0.0
    scale = k * abs(alpha) * amax * bmax + abs(beta) * cmax
    err = float(np.abs(got - want).max()) if got.size else 0.0
    if scale == 0.0:
        return 0.0 if err == 0.0 else float("inf")
    return err / (eps * scale)


def make_problem(m, n, k, kind="uniform", dtype="f32", c_kind="uniform", seed_base=0,
                 lda=None, ldb=None, ldc=None, int_range=(-3, 3), fill=float("nan")):
    """CPU tensors (A, B, C) plus their padded storages.  A, B in the
    operand dtype; C fp32.  Padded storages have NaN in the ld tail."""
    tdt = TORCH_DT[dtype]
    kw = dict(lo=int_range[0], hi=int_range[1]) if kind == "integers" else {}
    A = inputs.make(kind, m, k, inputs.SEED_A + seed_base, dtype=tdt, **kw)
    Bm = inputs.make(kind, k, n, inputs.SEED_B + seed_base, dtype=tdt, **kw)
    ckw = dict(lo=int_range[0], hi=int_range[1]) if c_kind == "integers" else {}
    C = inputs.make(c_kind, m, n, inputs.SEED_C + seed_base, dtype=torch.float32, **ckw)
    return dict(A=A, B=Bm, C=C, lda=lda or max(k, 1), ldb=ldb or max(n, 1), ldc=ldc or max(n, 1),
                fill=fill)


def to_device(prob, device="cuda"):
    """Device storages (padded with the poison value) and logical views."""
    out = {}
    for name, ld in (("A", prob["lda"]), ("B", prob["ldb"]), ("C", prob["ldc"])):
        x = prob[name]
        st, view = inputs.padded(x, ld, fill=prob["fill"]) if ld != x.shape[1] else (x.clone(), None)
        st = st.to(device)
        view = st[:, : x.shape[1]] if view is not None else st
        out[name] = view
        out[name + "_storage"] = st
    return out


def stratified_entries(m, n, levels, seed, tile=256, lanes_tiles=3):
    """(rows, cols) covering every tile x tile square of every C block of the
    library's levels-level partition with one random entry each, the four
    corners of every block, and complete 32 x 32 accumulator blocks (every
    lane and register of the MFMA output layout) at the first, a middle and
    the last tile of the grid: a wrong tile, a wrong block or a wrong lane
    position cannot escape."""
    import paper_1808_07984_amd as sg
    info = sg.plan_info(m, n, 1, levels)
    sm, sn, d = info.sub_m, info.sub_n, info.blocks_per_dim
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    tiles = []
    for R in range(d):
        r0, r1 = R * sm, min((R + 1) * sm, m)
        for Cc in range(d):
            c0, c1 = Cc * sn, min((Cc + 1) * sn, n)
            if r0 >= r1 or c0 >= c1:
                continue
            for tr in range(r0, r1, tile):
                for tc in range(c0, c1, tile):
                    tiles.append((tr, tc))
                    rows.append(rng.integers(tr, min(tr + tile, r1)))
                    cols.append(rng.integers(tc, min(tc + tile, c1)))
            rows += [r0, r0, r1 - 1, r1 - 1]
            cols += [c0, c1 - 1, c0, c1 - 1]
    for (tr, tc) in (tiles[0], tiles[len(tiles) // 2], tiles[-1])[:lanes_tiles]:
        rr, cc = np.meshgrid(np.arange(tr, min(tr + 32, m)), np.arange(tc, min(tc + 32, n)), indexing="ij")
        rows += rr.ravel().tolist()
        cols += cc.ravel().tolist()
    return np.asarray(rows, dtype=np.int64), np.asarray(cols, dtype=np.int64)
