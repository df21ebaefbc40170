"""Seeded synthetic inputs for the CC3 triples residual.

This module only draws random numbers; it holds none of the method's arithmetic.
Both the HIP path (through its tests and benchmark) and the CPU oracle are fed
from here, so they see identical inputs.

Recipe (stands in for the real molecules of the paper's application section,
whose integrals are not available): canonical orbital energies with occupied
values uniform in [-2.0, -0.5] and virtual values uniform in [0.2, 3.0], both
sorted ascending; Cholesky vectors L[J][p][q] drawn N(0, 0.05^2) and made
symmetric in (p, q) by mirroring the upper triangle; singles t1[i][a] drawn
N(0, (1e-3)^2); doubles t2[i][j][a][b] drawn N(0, (1e-2)^2) and made to obey
the pair symmetry t2[i][j][a][b] = t2[j][i][b][a] by keeping the draw at the
lexicographically smaller (i,a) <= (j,b) element.  Draw order: eps_occ, eps_vir,
L, t1, t2.  All arrays are float64 and C-contiguous.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 200701088


def _rng(no: int, nv: int, nchol: int, tag: int) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, int(no), int(nv), int(nchol), int(tag)])


def mirror_pairs(x: np.ndarray) -> np.ndarray:
    """Return t2 with t2[i][j][a][b] == t2[j][i][b][a], keeping the (i,a) <= (j,b) draw."""
    no, _, nv, _ = x.shape
    i = np.arange(no)[:, None, None, None]
    j = np.arange(no)[None, :, None, None]
    a = np.arange(nv)[None, None, :, None]
    b = np.arange(nv)[None, None, None, :]
    keep = (i < j) | ((i == j) & (a <= b))
    return np.ascontiguousarray(np.where(keep, x, x.transpose(1, 0, 3, 2)))


def mirror_cholesky(x: np.ndarray) -> np.ndarray:
    """Return L with L[J][q][p] == L[J][p][q], keeping the upper triangle (p <= q)."""
    up = np.triu(x)
    return np.ascontiguousarray(up + np.triu(x, 1).transpose(0, 2, 1))


def make_inputs(no: int, nv: int, nchol: int, tag: int = 0, t1_zero: bool = False) -> dict:
    """Seeded inputs {eps, L, t1, t2} for one residual call of size (no, nv, nchol)."""
    if no < 1 or nv < 1 or nchol < 1:
        raise ValueError("sizes must be positive")
    g = _rng(no, nv, nchol, tag)
    eps_o = np.sort(g.uniform(-2.0, -0.5, size=no))
    eps_v = np.sort(g.uniform(0.2, 3.0, size=nv))
    nmo = no + nv
    L = mirror_cholesky(g.normal(0.0, 0.05, size=(nchol, nmo, nmo)))
    t1 = g.normal(0.0, 1e-3, size=(no, nv))
    t2 = mirror_pairs(g.normal(0.0, 1e-2, size=(no, no, nv, nv)))
    if t1_zero:
        t1 = np.zeros_like(t1)
    return {
        "no": no, "nv": nv, "nchol": nchol,
        "eps": np.ascontiguousarray(np.concatenate([eps_o, eps_v])),
        "L": L, "t1": np.ascontiguousarray(t1), "t2": t2,
    }


def make_left_inputs(no: int, nv: int, tag: int = 0) -> dict:
    """Seeded left-state amplitudes for the transition-density contributions: an
    excitation energy omega uniform in [0.2, 0.6] (below every triples excitation of
    make_inputs' orbital energies, which start at 2.1), l1[i][a] ~ N(0, 0.05^2) and
    l2[i][j][a][b] ~ N(0, (1e-2)^2) with the pair symmetry of t2.  Draw order: omega,
    l1, l2."""
    if no < 1 or nv < 1:
        raise ValueError("sizes must be positive")
    g = np.random.default_rng([SEED_BASE, 13, int(no), int(nv), int(tag)])
    omega = float(g.uniform(0.2, 0.6))
    l1 = g.normal(0.0, 0.05, size=(no, nv))
    l2 = mirror_pairs(g.normal(0.0, 1e-2, size=(no, no, nv, nv)))
    return {"omega": omega, "l1": np.ascontiguousarray(l1), "l2": l2}


def perturb_t2(t2: np.ndarray, seed: int, scale: float = 1e-4) -> np.ndarray:
    """A solver-iteration-like update: t2 + N(0, scale^2), pair symmetry kept."""
    g = np.random.default_rng([SEED_BASE, 7, int(seed)])
    return mirror_pairs(t2 + g.normal(0.0, scale, size=t2.shape))


def sample_triples(no: int, count: int, seed: int = 0) -> np.ndarray:
    """A seeded uniform sample (without replacement) of unordered occupied triples
    i >= j >= k, excluding i == j == k, returned as int32 [count][3]."""
    allt = [(i, j, k) for i in range(no) for j in range(i + 1) for k in range(j + 1)
            if not (i == j == k)]
    g = np.random.default_rng([SEED_BASE, 11, int(no), int(seed)])
    count = min(count, len(allt))
    idx = np.sort(g.choice(len(allt), size=count, replace=False))
    return np.ascontiguousarray(np.array([allt[t] for t in idx], dtype=np.int32).reshape(-1, 3))


def _torch_gen(device, *key):
    import torch
    h = np.random.SeedSequence([SEED_BASE, *[int(k) for k in key]]).generate_state(1, np.uint64)[0]
    g = torch.Generator(device=device)
    g.manual_seed(int(h) & ((1 << 63) - 1))
    return g


def mirror_pairs_torch(x):
    """torch form of mirror_pairs (same element choice), on x's device."""
    import torch
    no, _, nv, _ = x.shape
    i = torch.arange(no, device=x.device).view(no, 1, 1, 1)
    j = torch.arange(no, device=x.device).view(1, no, 1, 1)
    a = torch.arange(nv, device=x.device).view(1, 1, nv, 1)
    b = torch.arange(nv, device=x.device).view(1, 1, 1, nv)
    keep = (i < j) | ((i == j) & (a <= b))
    return torch.where(keep, x, x.permute(1, 0, 3, 2)).contiguous()


def make_inputs_device(no: int, nv: int, nchol: int, tag: int = 0, device="cuda:0") -> dict:
    """The recipe of make_inputs drawn with torch's generator directly on `device`
    (for large batches of molecules; values differ from make_inputs, the
    distributions and symmetries are the same)."""
    import torch
    g = _torch_gen(device, 3, no, nv, nchol, tag)
    f64 = dict(dtype=torch.float64, device=device)
    eps_o = torch.sort(torch.rand(no, generator=g, **f64) * 1.5 - 2.0).values
    eps_v = torch.sort(torch.rand(nv, generator=g, **f64) * 2.8 + 0.2).values
    nmo = no + nv
    x = torch.randn(nchol, nmo, nmo, generator=g, **f64) * 0.05
    up = torch.triu(x)
    L = (up + torch.triu(x, 1).transpose(1, 2)).contiguous()
    t1 = (torch.randn(no, nv, generator=g, **f64) * 1e-3).contiguous()
    t2 = mirror_pairs_torch(torch.randn(no, no, nv, nv, generator=g, **f64) * 1e-2)
    return {"no": no, "nv": nv, "nchol": nchol, "eps": torch.cat([eps_o, eps_v]).contiguous(),
            "L": L, "t1": t1, "t2": t2}


def perturb_t2_device(t2, seed: int, scale: float = 1e-4):
    """torch form of perturb_t2 on t2's device (a solver-iteration-like update)."""
    import torch
    g = _torch_gen(t2.device, 7, seed)
    noise = torch.randn(t2.shape, generator=g, dtype=t2.dtype, device=t2.device) * scale
    return mirror_pairs_torch(t2 + noise)


def serving_mix(count: int = 64, seed: int = 5) -> list:
    """(no, nv, nchol) of `count` molecules: no uniform in [5, 20], nv uniform in
    [60, 250] (integers), Cholesky rank round(3 (no + nv))."""
    g = np.random.default_rng([SEED_BASE, 5, int(seed)])
    out = []
    for _ in range(count):
        no = int(g.integers(5, 21))
        nv = int(g.integers(60, 251))
        out.append((no, nv, int(round(3 * (no + nv)))))
    return out


def poisson_arrivals(count: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    g = np.random.default_rng([SEED_BASE, 6, int(seed)])
    return np.cumsum(g.exponential(1.0 / rate, size=count)) - 0.0
