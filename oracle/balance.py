"""Run-time balanced energy split (Fig. 1b), test oracle.

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline use this package.

The paper balances the windows so that all of them finish the first
Wang-Landau iteration after about the same number of MC steps, and says the
split can be estimated from the first-iteration data of a short pre-run with
equal windows.  The reading implemented here (plain Python, one bin at a
time):

1. A pre-run window v whose first iteration took S_v MC steps per walker
   gets the cost width S_v ** (1 / alpha) (alpha = 2: a random walk needs a
   time quadratic in the range it covers); its cost density is that width
   divided by its number of bins.
2. Bin b's density c_b is the average density of the pre-run windows that
   contain b.
3. The centre of bin b sits at x_b = c_0 + ... + c_{b-1} + c_b / 2.
4. The h new windows are the equal-size split of Fig. 1a done in x:
   width W = (x_last - x_0) / (1 + (h - 1)(1 - o)); window i spans
   [x_0 + i (1 - o) W, that + W]; each end goes to the bin whose centre is
   closest (a tie goes to the higher bin).
5. Repairs, window by window from the low end: the first window starts at
   bin 0 and the last ends at the last bin; a window starts after the
   previous one starts and at least 4 bins before the previous one ends (so
   neighbours share >= 5 bins, what the five-point join needs), ends after
   the previous one ends, and is at least 5 bins wide.  A repair that would
   leave the bin range, or cannot keep the starts increasing, is an error.
"""
import math


def balanced_windows(nbins, h, overlap, pre_lo, pre_hi, pre_steps, alpha=2.0):
    """Returns (lo, hi) lists of h inclusive bin edges; raises ValueError."""
    on, od = overlap
    if nbins < 5 or h < 1 or not (0 <= on < od) or not alpha > 0:
        raise ValueError("bad arguments")
    total = [0.0] * nbins
    count = [0] * nbins
    for a, b, S in zip(pre_lo, pre_hi, pre_steps):
        if not (0 <= a <= b < nbins) or not S > 0:
            raise ValueError("bad pre-run window")
        dens = math.pow(S, 1.0 / alpha) / (b - a + 1)
        for j in range(a, b + 1):
            total[j] += dens
            count[j] += 1
    centres = []
    run = 0.0
    for j in range(nbins):
        if count[j] == 0:
            raise ValueError(f"bin {j} is in no pre-run window")
        c = total[j] / count[j]
        centres.append(run + 0.5 * c)
        run = run + c
    frac = (od - on) / od
    width = (centres[-1] - centres[0]) / (1.0 + (h - 1) * frac)

    def closest(v):
        best = 0
        for j in range(1, nbins):
            dj, db = abs(centres[j] - v), abs(centres[best] - v)
            if dj <= db:
                best = j
        return best

    lo, hi = [], []
    for i in range(h):
        start = centres[0] + i * frac * width
        lo.append(closest(start))
        hi.append(closest(start + width))
    lo[0], hi[-1] = 0, nbins - 1
    for i in range(h):
        if i > 0:
            lo[i] = max(lo[i], lo[i - 1] + 1)
            lo[i] = min(lo[i], hi[i - 1] - 4)
            if lo[i] <= lo[i - 1]:
                raise ValueError("too many windows for the bins")
            hi[i] = max(hi[i], hi[i - 1] + 1)
        hi[i] = max(hi[i], lo[i] + 4)
        if hi[i] > nbins - 1:
            raise ValueError("too many windows for the bins")
    return lo, hi
