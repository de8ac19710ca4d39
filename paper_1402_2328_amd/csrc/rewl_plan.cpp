// Run-time balanced energy split (Fig. 1b of the paper): window edges chosen
// so that every window finishes its first Wang-Landau iteration after about
// the same number of MC steps, estimated from a short pre-run with any split
// (normally the equal-size one of Fig. 1a).  Host code only.
//
// Cost model.  A window whose first iteration took S MC steps per walker is
// given a cost width S^(1/alpha) (alpha = 2: a random walk needs a time that
// grows with the square of the range it must cover), spread evenly over its
// bins.  A bin's cost density is the mean density of the pre-run windows
// that contain it.  With x_b the cost coordinate of the centre of bin b
// (cumulative density up to b plus half of b's own), the new windows are the
// equal split of Fig. 1a carried out in x: h windows of width
// W = (x_last - x_first) / (1 + (h-1)(1-o)), window i starting at
// x_first + i (1-o) W; each edge is mapped to the bin whose centre is
// nearest (ties to the higher bin).  Fix-ups keep every window at least five
// bins wide and every neighbour overlap at least five bins (the joining
// stencil of Sec. 3 needs that much), edges strictly increasing.
#include <math.h>
#include <stdint.h>

#include <vector>

#include "rewl.h"

namespace {

int nearest_centre(const std::vector<double>& x, double v) {
  // first centre >= v, then compare with its left neighbour
  int lo = 0, hi = (int)x.size() - 1;
  if (v <= x[0]) return 0;
  if (v >= x[hi]) return hi;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (x[mid] < v) lo = mid;
    else hi = mid;
  }
  // x[lo] < v <= x[hi]
  return (v - x[lo] < x[hi] - v) ? lo : hi;
}

}  // namespace

extern "C" int rewl_balanced_windows(int32_t nbins, int32_t h, int32_t overlap_num,
                                     int32_t overlap_den, int32_t pre_h, const int32_t* pre_lo,
                                     const int32_t* pre_hi, const double* pre_steps, double alpha,
                                     int32_t* lo, int32_t* hi) {
  if (nbins < 5 || h < 1 || pre_h < 1 || !pre_lo || !pre_hi || !pre_steps || !lo || !hi)
    return REWL_E_INVAL;
  if (overlap_den <= 0 || overlap_num < 0 || overlap_num >= overlap_den) return REWL_E_INVAL;
  if (!(alpha > 0.0) || !isfinite(alpha)) return REWL_E_INVAL;
  std::vector<double> dens_sum(nbins, 0.0);
  std::vector<int32_t> cover(nbins, 0);
  for (int v = 0; v < pre_h; ++v) {
    if (pre_lo[v] < 0 || pre_hi[v] >= nbins || pre_hi[v] < pre_lo[v]) return REWL_E_INVAL;
    if (!(pre_steps[v] > 0.0) || !isfinite(pre_steps[v])) return REWL_E_INVAL;
    const double d = pow(pre_steps[v], 1.0 / alpha) / (double)(pre_hi[v] - pre_lo[v] + 1);
    for (int b = pre_lo[v]; b <= pre_hi[v]; ++b) {
      dens_sum[b] += d;
      cover[b] += 1;
    }
  }
  std::vector<double> x(nbins);
  double acc = 0.0;
  for (int b = 0; b < nbins; ++b) {
    if (cover[b] == 0) return REWL_E_INVAL;
    const double c = dens_sum[b] / (double)cover[b];
    x[b] = acc + 0.5 * c;
    acc = acc + c;
  }
  const double step = (double)(overlap_den - overlap_num) / (double)overlap_den;
  const double W = (x[nbins - 1] - x[0]) / (1.0 + (double)(h - 1) * step);
  for (int i = 0; i < h; ++i) {
    const double start = x[0] + (double)i * step * W;
    lo[i] = nearest_centre(x, start);
    hi[i] = nearest_centre(x, start + W);
  }
  lo[0] = 0;
  hi[h - 1] = nbins - 1;
  // fix-ups, low to high: width >= 5 bins, strictly increasing edges,
  // overlap with the previous window >= 5 bins
  for (int i = 0; i < h; ++i) {
    if (i > 0) {
      if (lo[i] <= lo[i - 1]) lo[i] = lo[i - 1] + 1;
      if (lo[i] > hi[i - 1] - 4) lo[i] = hi[i - 1] - 4;
      if (lo[i] <= lo[i - 1]) return REWL_E_INVAL;
      if (hi[i] <= hi[i - 1]) hi[i] = hi[i - 1] + 1;
    }
    if (hi[i] < lo[i] + 4) hi[i] = lo[i] + 4;
    if (hi[i] > nbins - 1) return REWL_E_INVAL;
  }
  if (hi[h - 1] != nbins - 1) return REWL_E_INVAL;
  return REWL_OK;
}
