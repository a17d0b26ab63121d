"""Writes fft_plans_rows.inc and fft_plans_cols.inc: one FFT plan per
supported line length, for the row pass (x) and for the column passes (y, z).

The oversampled FFT of the type-3 path (paper section 2.2, step 2) runs, per
line of n1 = L modes, two L-point transforms (the even and odd outputs of the
zero-padded 2L-point transform).  A plan fixes, for one L:

  NL     lines per workgroup of 512 threads (for columns, row segments in
         global memory twice as long as with 256 threads, for the same work
         per thread); a power of two for columns, up to 128, so that short
         columns still give a workgroup enough work;
  LP     line stride in LDS: odd for rows; for columns 16/NL mod 16 (1 mod 16
         past 16 lines), so that the lines of 16 lanes (columns first) fall in
         distinct banks;
  F[g]   the radix of each group (2 to 16), prod F = L: group g is a Stockham
         step of radix F whose F-point DFT runs in registers, so a line goes
         through LDS only between groups.  Group g's L / F_g butterflies per
         line are dealt to the threads in rounds; a middle group holds every
         round's points in registers across its barrier (at most 24), the
         first group loads all of a thread's points before transforming them
         (at most 32), and the last group keeps its even-phase outputs in
         registers (at most 16) until the odd phase writes both;

The search minimises an estimate of the instructions per point -- the small
DFTs, the twiddle products, LDS and index work, counted over every round of
the workgroup's threads so that idle lanes cost, and for columns a fixed cost per
workgroup (its set-up and twiddle rows) spread over its points -- with a
penalty when the LDS a
workgroup holds leaves fewer than 16 wavefronts per compute unit (the passes
wait on memory and barriers), and a small one per group (one barrier pair
each), and the LDS accesses of every group are weighted by their bank-conflict
degree, simulated for the first wavefront with the kernel's lane orders
(the first group of the row pass writes at lane stride F_0, for example,
which meets every bank only when F_0 is odd).
Run by build.py before compiling.
"""
import math
import os
import sys

TPB_ROWS, TPB_COLS = 512, 512
# LDS per workgroup: 16 wavefronts per compute unit (two workgroups)
LDS_CAP_ROWS, LDS_CAP_COLS = 80 * 1024, 80 * 1024
LDS_CU = 160 * 1024
RADICES = (2, 3, 4, 5, 6, 8, 9, 10, 12, 15, 16)
GMAX, GMAX_HARD = 4, 6
HOLD = 24      # points a middle group holds across its barrier
HOLD_IN = 32   # points a thread loads before its first DFT
HOLD_OUT = 16  # even-phase outputs kept until the odd phase stores both
# Column plans stop at 2304 points.  With 256-thread workgroups and a 40 KB
# cap a 2250-point column workgroup held one line (8-byte segments per row),
# and the y pass of the 3-D disk workload took 75 ms against 60 ms with the
# general kernel; with 512 threads and 80 KB it holds two lines, and that pass
# takes 51 ms against 58.  Rows are contiguous, so their plans go on to 4608
# points (one row per workgroup past 3600).
LMIN, LMAX = 16, 2304
LMAX_ROWS = 4608

# real operations per point of a small DFT (additions and multiplications,
# a fused multiply-add counted once)
BASE = {2: 2.0, 3: 4.7, 4: 4.0, 5: 7.2}


def smooth(n: int) -> bool:
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def split(F: int) -> int:
    """The first factor of a composite small DFT (as fft_reg.h splits it)."""
    if F % 4 == 0 and F > 4:
        return 4
    for a in (2, 3, 5):
        if F % a == 0:
            return a
    raise ValueError(F)


def dft_cost(F: int) -> float:
    if F in BASE:
        return BASE[F]
    a = split(F)
    b = F // a
    return dft_cost(a) + dft_cost(b) + 4.0 * (a - 1) * (b - 1) / F


def sequences(L: int, gmax: int):
    out = []

    def rec(rem, acc):
        if rem == 1:
            if len(acc) >= 2:
                out.append(tuple(acc))
            return
        if len(acc) >= gmax:
            return
        for d in RADICES:
            if rem % d == 0:
                rec(rem // d, acc + [d])

    rec(L, [])
    return out


COL_NL = (1, 2, 4, 8, 16, 32, 64, 128)
COL_WG_FIXED = TPB_COLS * 40.0  # per-workgroup set-up of a column plan, in the cost's units


def line_stride(L: int, NL: int, cols: bool) -> int:
    if not cols:
        return L + 1 if L % 2 == 0 else L
    want = (16 // NL) % 16 if NL <= 16 else 1
    n = L
    while n % 16 != want:
        n += 1
    return n


def twiddle_entries(Fs) -> int:
    """Entries of the twiddle rows (fft_reg.h, Plan::TW)."""
    G = len(Fs)
    tot, p = 0, Fs[0]
    for g in range(1, G):
        W = Fs[g] if g == G - 1 else Fs[g] - 1
        S = W if W % 2 == 1 else W + 1
        tot += p * S
        p *= Fs[g]
    return tot


def conflicts(addrs) -> float:
    """LDS cycles per 16-lane group for 8-byte accesses, relative to a
    conflict-free access: the largest number of distinct addresses that
    share a bank pair (32 four-byte banks), averaged over the groups."""
    tot, n = 0.0, 0
    for g0 in range(0, len(addrs), 16):
        seen = {}
        for a in addrs[g0:g0 + 16]:
            if a is None:
                continue
            seen.setdefault(a % 16, set()).add(a)
        if seen:
            tot += max(len(v) for v in seen.values())
            n += 1
    return tot / n if n else 1.0


def lds_conflict_factor(L: int, NL: int, LP: int, Fs, cols: bool) -> float:
    """Average conflict degree of the LDS writes and reads of every group, for
    the first wavefront of a workgroup, with the lane orders of fft_reg.h."""
    G = len(Fs)
    p = 1
    tot, cnt = 0.0, 0
    for g, F in enumerate(Fs):
        Q = L // F
        across = cols and g in (0, G - 1)
        lanes = []
        for b in range(64):
            if b >= NL * Q:
                lanes.append(None)
                continue
            l, i = (b % NL, b // NL) if across else (b // Q, b % Q)
            lanes.append((l, i))
        for j in range(F):
            if g > 0:  # reads of group g at i + j Q
                tot += conflicts([None if x is None else x[0] * LP + x[1] + j * Q for x in lanes])
                cnt += 1
            if g < G - 1:  # writes to (i div p) p F + (i mod p) + j p
                tot += conflicts([None if x is None else x[0] * LP + (x[1] // p) * p * F + x[1] % p + j * p
                                  for x in lanes])
                cnt += 1
        p *= F
    return tot / cnt if cnt else 1.0


def plan(L: int, cols: bool, gmax: int = GMAX):
    TPB = TPB_COLS if cols else TPB_ROWS
    LDS_CAP = LDS_CAP_COLS if cols else LDS_CAP_ROWS
    best = None
    for Fs in sequences(L, gmax):
        G = len(Fs)
        for NL in (COL_NL if cols else range(1, 33)):
            LP = line_stride(L, NL, cols)
            lds = (NL * LP + twiddle_entries(Fs)) * 8
            if lds > LDS_CAP:
                break
            R = [math.ceil(NL * (L // F) / TPB) for F in Fs]
            if max([R[g] * Fs[g] for g in range(1, G - 1)] or [0]) > HOLD:
                continue
            # registers: the first group's loads in flight, and the last
            # group's even-phase outputs kept through the odd phase
            if R[0] * Fs[0] > HOLD_IN or R[-1] * Fs[-1] > HOLD_OUT:
                continue
            work = 0.0
            for g, F in enumerate(Fs):
                per = F * dft_cost(F) + 2.0 * F + 6.0  # DFT, two LDS accesses per point, indices
                if g > 0:
                    per += 4.0 * (F - 1) + (4.0 if g == G - 1 else 0.0)  # twiddle products
                if g == G - 1:
                    per += 1.5 * F  # output window and addresses
                work += R[g] * TPB * per
            cost = (work + (COL_WG_FIXED if cols else 0.0)) / (NL * L)
            waves = min(LDS_CU // lds, 2048 // TPB) * TPB // 64
            # LDS accesses (two per point and group boundary) at their conflict degree
            lds_cost = 2.0 * (G - 1) * 2.0 * lds_conflict_factor(L, NL, LP, Fs, cols)
            score = (cost + lds_cost) * max(1.0, 16.0 / waves) + 3.0 * G
            key = (round(score, 3), 0 if Fs[0] % 2 else 1, G)
            if best is None or key < best[0]:
                best = (key, (L, NL, LP) + Fs + (1,) * (GMAX_HARD - G))
    if best is None and gmax < GMAX_HARD:
        return plan(L, cols, GMAX_HARD)
    return None if best is None else best[1]


def main(directory: str) -> None:
    for cols, name in ((False, "fft_plans_rows.inc"), (True, "fft_plans_cols.inc")):
        lines = ["// Generated by gen_fft_plans.py: FV_FFT_PLAN(L, NL, LP, F1, F2, F3, F4, F5, F6)"]
        for L in range(LMIN, (LMAX if cols else LMAX_ROWS) + 1, 2):
            if not smooth(L):
                continue
            p = plan(L, cols)
            if p is not None:
                lines.append("FV_FFT_PLAN(" + ", ".join(str(v) for v in p) + ")")
        text = "\n".join(lines) + "\n"
        path = os.path.join(directory, name)
        if not os.path.exists(path) or open(path).read() != text:
            with open(path, "w") as f:
                f.write(text)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.dirname(os.path.abspath(__file__)))
