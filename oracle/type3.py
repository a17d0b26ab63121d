"""Step-by-step FP64 type-3 NUFFT for visibilities, in numpy.

TEST INFRASTRUCTURE ONLY (oracle side; the product never imports this).

This is the slow, plain counterpart of the three stages the paper describes
for the type-3 transform (section 2.2, enumerated steps 1-3, the grid-size
equation and the centring remark that follows it), used to check the GPU
path stage by stage.  The end result is itself pinned to the direct sum
(oracle.direct_vis) within the requested eps in the tests.

Readings of the paper taken here (each one listed in the design doc):
  * target modes x_k = -2 pi nu b_k / c, sources s_j = (l, m[, n]);
  * both point sets are translated to boxes centred on zero (section 2.2,
    after the grid-size equation): s_c, S from the source bounding box,
    x_c, X from the target bounding box; X is an angular frequency
    (radians), so X*S is dimensionless;
  * w = ceil(log10(1/eps)) + 2 points per dimension (the paper's rule plus
    one), beta = 2.3 w, sigma = 2;
  * n1 = ceil((2 sigma / pi) X S + w) rounded up to an even {2,3,5}-smooth
    size is the spreading grid, n2 = sigma n1 the FFT grid;
  * the deconvolution is done twice, as the type-3 algorithm needs: by the
    kernel transform at the uniform modes before the FFT, and at the
    non-uniform targets after interpolation;
  * real strengths give V(-b) = conj V(b), so targets are reflected into the
    half-space b_a >= 0 of the axis a with the largest extent (ties and
    zeros broken by the next axes' signs), then conjugated back.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

from .es_kernel import es_beta, es_phi, es_phihat

C_LIGHT = 299792458.0
SIGMA = 2.0


def kernel_width(eps: float) -> int:
    """Points per dimension touched by the kernel: ceil(log10(1/eps)) + 2, in [2, 16]."""
    w = int(math.ceil(-math.log10(eps) - 1e-9)) + 2
    return max(2, min(16, w))


def next_smooth_even(n: int) -> int:
    """Smallest even integer >= n whose only prime factors are 2, 3 and 5."""
    n = max(2, int(n))
    if n % 2:
        n += 1
    while True:
        m = n
        for p in (2, 3, 5):
            while m % p == 0:
                m //= p
        if m == 1:
            return n
        n += 2


def fold_targets(b: np.ndarray, axis: int):
    """Reflect baselines into b[axis] >= 0 (ties broken by the remaining axes
    in order).  Returns (folded baselines, bool flag 'was reflected').
    axis = -1: no folding (the paper's plain targets)."""
    d = b.shape[1]
    if axis < 0:
        return b.copy(), np.zeros(b.shape[0], dtype=bool)
    order = [axis] + [a for a in range(d) if a != axis]
    flip = np.zeros(b.shape[0], dtype=bool)
    decided = np.zeros(b.shape[0], dtype=bool)
    for a in order:
        neg = (~decided) & (b[:, a] < 0)
        pos = (~decided) & (b[:, a] > 0)
        flip |= neg
        decided |= neg | pos
    return np.where(flip[:, None], -b, b), flip


@dataclass
class Plan:
    dim: int
    w: int
    beta: float
    s_c: np.ndarray
    S: np.ndarray          # effective half-widths of the source box
    b_c: np.ndarray        # centre of the folded baseline box (metres)
    B: np.ndarray          # half-widths of the folded baseline box (metres)
    fold_axis: int
    n1: List[np.ndarray] = field(default_factory=list)   # per frequency, [dim]
    X: List[np.ndarray] = field(default_factory=list)    # per frequency effective X (rad)
    x_c: List[np.ndarray] = field(default_factory=list)  # per frequency target centre (rad)

    def n2(self, f: int) -> np.ndarray:
        return (SIGMA * self.n1[f]).astype(np.int64)


def baselines(ant: np.ndarray) -> np.ndarray:
    """b_ij = x_i - x_j for i <= j, row-major."""
    i, j = np.triu_indices(ant.shape[0])
    return ant[i] - ant[j]


def make_plan(ant: np.ndarray, src: np.ndarray, freq: np.ndarray, eps: float, dim: int, fold: bool = True) -> Plan:
    """fold=False keeps the targets as the paper states them (section 2.2, the
    type-3 targets): no reflection into a half-space, fold_axis = -1."""
    w = kernel_width(eps)
    s = src[:, :dim]
    b = baselines(ant)[:, :dim]
    if s.shape[0]:
        smin, smax = s.min(0), s.max(0)
    else:
        smin = smax = np.zeros(dim)
    s_c = 0.5 * (smin + smax)
    S = 0.5 * (smax - smin)
    ext = b.max(0) - b.min(0)
    axis = int(np.argmax(ext * np.maximum(S, 1e-300))) if fold else -1
    bf, _ = fold_targets(b, axis)
    bmin, bmax = bf.min(0), bf.max(0)
    b_c = 0.5 * (bmin + bmax)
    B = 0.5 * (bmax - bmin)
    plan = Plan(dim=dim, w=w, beta=es_beta(w), s_c=s_c, S=S.copy(), b_c=b_c, B=B, fold_axis=axis)
    for nu in freq:
        k = 2.0 * math.pi * nu / C_LIGHT
        X = np.maximum(k * B, 1.0)
        Se = np.maximum(S, 1.0 / X)
        n1 = np.array([next_smooth_even(math.ceil(2.0 * SIGMA / math.pi * X[a] * Se[a] + w))
                       for a in range(dim)], dtype=np.int64)
        plan.n1.append(n1)
        plan.X.append(X)
        plan.x_c.append(-k * b_c)
    return plan


def spread(plan: Plan, f: int, src: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Step 1 (spreading) for frequency index f, then the first deconvolution.

    Returns b~ on the n1 grid, axes ordered (.., y, x) with mode index
    m = l - n1/2 along each axis.  c are the real strengths beam*flux."""
    d, w, beta = plan.dim, plan.w, plan.beta
    n1, X = plan.n1[f], plan.X[f]
    s = src[:, :d]
    # pre-phase by the target-box centre: c'_j = c_j exp(i x_c . (s_j - s_c))
    cp = c.astype(np.complex128) * np.exp(1j * ((s - plan.s_c) @ plan.x_c[f]))
    grid = np.zeros(tuple(int(v) for v in n1[::-1]), dtype=np.complex128)
    l0, wts = [], []
    for a in range(d):
        g = n1[a] / 2.0 + (s[:, a] - plan.s_c[a]) * SIGMA * X[a] / math.pi
        first = np.ceil(g - w / 2.0).astype(np.int64)
        first = np.clip(first, 0, n1[a] - w)
        l0.append(first)
        wts.append(es_phi((first[:, None] + np.arange(w)[None, :] - g[:, None]) / (w / 2.0), beta))
    for j in range(s.shape[0]):
        block = cp[j]
        for a in range(d):
            block = np.multiply.outer(wts[a][j], block) if a else wts[a][j] * block
        # block axes are (x) for d=1 .. built as (a_{d-1}, ..., a_0): outer puts the new axis first
        sl = tuple(slice(int(l0[a][j]), int(l0[a][j]) + w) for a in reversed(range(d)))
        grid[sl] += block
    # deconvolution at the uniform modes: divide by prod_a psi2hat(m_a)
    for a in range(d):
        n2a = SIGMA * n1[a]
        alpha2 = w * math.pi / n2a
        m = np.arange(n1[a]) - n1[a] // 2
        p2 = alpha2 * es_phihat(alpha2 * m, beta)
        shape = [1] * d
        shape[d - 1 - a] = int(n1[a])
        grid = grid / p2.reshape(shape)
    return grid


def fft_upsampled(plan: Plan, f: int, bt: np.ndarray) -> np.ndarray:
    """Step 2: zero-pad mode m to index (m mod n2) and take
    g_p = sum_m b~_m exp(+i m p 2 pi / n2) along every axis (full n2 grid)."""
    d = plan.dim
    n1 = plan.n1[f]
    n2 = plan.n2(f)
    big = np.zeros(tuple(int(v) for v in n2[::-1]), dtype=np.complex128)
    idx = [((np.arange(n1[a]) - n1[a] // 2) % n2[a]) for a in reversed(range(d))]
    big[np.ix_(*idx)] = bt
    return np.fft.ifftn(big) * float(np.prod(n2))


def interp_and_correct(plan: Plan, f: int, g: np.ndarray, freq_hz: float, b: np.ndarray) -> np.ndarray:
    """Step 3: interpolate the FFT grid at each target with the kernel, divide
    by the kernel transform at the target, apply the centring phase
    exp(i x_k . s_c), and undo the reflection by conjugation."""
    d, w, beta = plan.dim, plan.w, plan.beta
    n1, n2, X = plan.n1[f], plan.n2(f), plan.X[f]
    bf, flip = fold_targets(b[:, :d], plan.fold_axis)
    k = 2.0 * math.pi * freq_hz / C_LIGHT
    x = -k * bf
    xp = x - plan.x_c[f]
    acc = np.zeros(b.shape[0], dtype=np.complex128)
    p0, wts = [], []
    fac = np.ones(b.shape[0], dtype=np.complex128)
    for a in range(d):
        q = (n1[a] / 2.0) * xp[:, a] / X[a]
        first = np.ceil(q - w / 2.0).astype(np.int64)
        p0.append(first)
        wts.append(es_phi((first[:, None] + np.arange(w)[None, :] - q[:, None]) / (w / 2.0), beta))
        h, h2 = 2.0 * math.pi / n1[a], 2.0 * math.pi / n2[a]
        alpha1 = w * h / 2.0
        kappa = (n1[a] / (2.0 * SIGMA * X[a])) * xp[:, a]
        fac *= h * h2 / (alpha1 * es_phihat(alpha1 * kappa, beta))
    for t in range(b.shape[0]):
        # gather the w^d neighbourhood with periodic wrap
        ix = [np.mod(p0[a][t] + np.arange(w), n2[a]) for a in range(d)]
        sub = g[np.ix_(*[ix[a] for a in reversed(range(d))])]
        wt = wts[0][t]
        for a in range(1, d):
            wt = np.multiply.outer(wts[a][t], wt)
        val = np.sum(sub * wt)
        acc[t] = val
    fac *= np.exp(1j * (x @ plan.s_c))
    v = acc * fac
    return np.where(flip, np.conj(v), v)


def type3_vis(ant: np.ndarray, src: np.ndarray, freq: np.ndarray, c: np.ndarray, eps: float,
              dim: int, pairs: np.ndarray | None = None, fold: bool = True) -> np.ndarray:
    """Whole type-3 pipeline for every frequency.  c: [n_freq, n_src] real.
    Returns complex128 [n_freq, n_out]."""
    plan = make_plan(ant, src, freq, eps, dim, fold)
    b = baselines(ant)
    if pairs is not None:
        b = b[pairs]
    out = np.zeros((len(freq), b.shape[0]), dtype=np.complex128)
    for f, nu in enumerate(freq):
        bt = spread(plan, f, src, c[f])
        g = fft_upsampled(plan, f, bt)
        out[f] = interp_and_correct(plan, f, g, nu, b)
    return out
