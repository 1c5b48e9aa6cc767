"""Seeded synthetic inputs shared by the tests and the benchmark.

This module only draws numbers; it holds none of the method's arithmetic.
Every generator uses a torch CPU generator seeded explicitly, so the GPU path
and the CPU oracle always see identical operands.

Distributions (the paper measures synthetic matrices and does not state their
values, Experiment section):
  uniform   i.i.d. U[-1, 1]
  normal    i.i.d. N(0, 1)
  integers  i.i.d. uniform over {lo..hi}, stored as floats (exactness checks)
  scaled    rows (of A) or columns (of B) rescaled so their 2-norms are
            10**u with u ~ U[-3, 3]: norms spread over 1e-3 .. 1e3

Leading dimensions: ``padded`` embeds a matrix in a wider row-major buffer and
fills the unused tail of every row with a poison value (NaN by default) so a
kernel that reads past the logical width is caught.
"""
import torch

SEED_A, SEED_B, SEED_C, SEED_DC = 0, 1, 2, 3


def _gen(seed):
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return g


def uniform(rows, cols, seed, dtype=torch.float32):
    return (torch.rand(rows, cols, generator=_gen(seed), dtype=torch.float32) * 2 - 1).to(dtype)


def normal(rows, cols, seed, dtype=torch.float32):
    return torch.randn(rows, cols, generator=_gen(seed), dtype=torch.float32).to(dtype)


def integers(rows, cols, seed, lo=-3, hi=3, dtype=torch.float32):
    x = torch.randint(lo, hi + 1, (rows, cols), generator=_gen(seed), dtype=torch.int32)
    return x.to(dtype)


def scaled(rows, cols, seed, axis=0, decades=3.0, dtype=torch.float32):
    """N(0,1) matrix whose rows (axis=0) or columns (axis=1) have 2-norms
    10**u, u ~ U[-decades, decades]."""
    g = _gen(seed)
    x = torch.randn(rows, cols, generator=g, dtype=torch.float64)
    nvec = rows if axis == 0 else cols
    u = (torch.rand(nvec, generator=g, dtype=torch.float64) * 2 - 1) * decades
    norms = x.norm(dim=1 - axis, keepdim=True).clamp_min(1e-300)
    scale = (10.0 ** u).reshape(-1, 1) if axis == 0 else (10.0 ** u).reshape(1, -1)
    return (x / norms * scale).to(dtype)


def padded(x, ld, fill=float("nan")):
    """Returns (storage, view): storage is rows x ld, view is the rows x cols
    logical matrix inside it (stride(0) == ld).  Columns cols..ld-1 hold
    `fill`."""
    rows, cols = x.shape
    if ld < cols:
        raise ValueError("ld %d < cols %d" % (ld, cols))
    storage = torch.full((rows, ld), fill, dtype=x.dtype, device=x.device)
    storage[:, :cols] = x
    return storage, storage[:, :cols]


def make(kind, rows, cols, seed, dtype=torch.float32, **kw):
    """Dispatch by distribution name."""
    if kind == "uniform":
        return uniform(rows, cols, seed, dtype)
    if kind == "normal":
        return normal(rows, cols, seed, dtype)
    if kind == "integers":
        return integers(rows, cols, seed, dtype=dtype, **kw)
    if kind == "scaled":
        return scaled(rows, cols, seed, dtype=dtype, **kw)
    if kind == "zeros":
        return torch.zeros(rows, cols, dtype=dtype)
    raise ValueError("unknown distribution %r" % (kind,))
