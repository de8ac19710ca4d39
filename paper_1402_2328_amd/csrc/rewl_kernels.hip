// REWL kernels for gfx950 (MI355X), everything except the sweep (which is
// in rewl_sweep.hip).
//
// Once per cycle: k_merge_windows (flatness by block reductions
// and the in-window average), k_merge_finish, k_exchange (Eq. 1, swaps
// configuration indices, never lattice data), k_exchange_finish.  End of
// run: k_join (Sec. 3 joining + normalisation in FP64), k_jackknife
// (error bars from the m pieces per window) and k_thermo (Sec. 5, Eqs. 7-8).
#include <float.h>
#include <math.h>

#include <mutex>

#include "rewl_device.h"
#include "rewl_internal.h"

namespace rewl {

namespace {

__device__ __forceinline__ int find_instance(const DevPtrs& P, int slot) {
  int i = 0;
  while (i + 1 < P.n_inst && P.inst[i + 1].slot_base <= slot) ++i;
  return i;
}

__device__ __forceinline__ uint4 draw(const InstDesc& I, uint64_t idx, uint32_t w2, uint32_t tag) {
  return philox10(make_uint4((uint32_t)idx, (uint32_t)(idx >> 32), w2,
                             tag | ((uint32_t)I.inst << 8)),
                  I.key0, I.key1);
}

__device__ int32_t full_energy(const InstDesc& I, const int8_t* sp) {
  const int L = I.L;
  int32_t e = 0;
  for (int y = 0; y < L; ++y) {
    const int yd = (y + 1 == L) ? 0 : y + 1;
    for (int x = 0; x < L; ++x) {
      const int xr = (x + 1 == L) ? 0 : x + 1;
      const int s0 = sp[y * L + x], sr = sp[y * L + xr], sd = sp[yd * L + x];
      if (I.model == kIsing) e -= s0 * sr + s0 * sd;
      else e -= (s0 == sr) + (s0 == sd);
    }
  }
  return e;
}

// Proposal on a lattice in global memory (warm-up only).
__device__ int propose_global(const InstDesc& I, const int8_t* sp, uint4 r, int& site, int& nv) {
  const int L = I.L;
  const int st = (int)__umulhi(r.x, (uint32_t)I.N);
  const int y = st / L, x = st - y * L;
  const int a = sp[y * L + ((x + 1 == L) ? 0 : x + 1)];
  const int b = sp[y * L + ((x == 0) ? L - 1 : x - 1)];
  const int c = sp[((y + 1 == L) ? 0 : y + 1) * L + x];
  const int d = sp[((y == 0) ? L - 1 : y - 1) * L + x];
  const int s0 = sp[st];
  site = st;
  if (I.model == kIsing) {
    nv = -s0;
    return 2 * s0 * (a + b + c + d);
  }
  int v = s0 + 1 + (int)__umulhi(r.y, (uint32_t)(I.q - 1));
  v = (v >= I.q) ? v - I.q : v;
  nv = v;
  return ((a == s0) + (b == s0) + (c == s0) + (d == s0)) - ((a == v) + (b == v) + (c == v) + (d == v));
}

__device__ __forceinline__ int32_t dist_to(int32_t E, int32_t elo, int32_t ehi) {
  return E < elo ? elo - E : (E > ehi ? E - ehi : 0);
}

}  // namespace

// ---------------------------------------------------------------------------
// Initialisation: random spins (one Philox block per 4 sites), full energy,
// then warm-up into the window: greedy moves that never increase the
// distance of E to the window, budget 1000 N; on failure one restart from an
// extreme state (ground state below the middle of the range, checkerboard
// above) and a second budget.  One thread per walker; not on the hot path.
// ---------------------------------------------------------------------------
__global__ void k_init(DevPtrs P) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= P.n_slots) return;
  const InstDesc I = P.inst[find_instance(P, g)];
  const int loc = g - I.slot_base;
  const int w = loc / I.m;
  const WinDesc W = P.win[I.win_base + w];
  int8_t* sp = P.spins + I.spin_base + (int64_t)loc * I.npad;
  for (int site = 0; site < I.N; site += 4) {
    const uint4 r = draw(I, (uint64_t)(site >> 2), (uint32_t)loc, kTagInit);
    const uint32_t rv[4] = {r.x, r.y, r.z, r.w};
    for (int j = 0; j < 4 && site + j < I.N; ++j) {
      const uint32_t v = rv[j];
      sp[site + j] = (I.model == kIsing) ? (int8_t)((v >> 31) ? 1 : -1)
                                         : (int8_t)__umulhi(v, (uint32_t)I.q);
    }
  }
  const int32_t elo = I.emin + W.lo * I.binw, ehi = I.emin + W.hi * I.binw;
  int32_t E = full_energy(I, sp);
  uint64_t wa = 0;
  for (int phase = 0; phase < 2; ++phase) {
    const int64_t budget = 1000LL * I.N;
    for (int64_t it = 0; it < budget && dist_to(E, elo, ehi) > 0; ++it) {
      const uint4 r = draw(I, wa++, (uint32_t)loc, kTagWarm);
      int site, nv;
      const int dE = propose_global(I, sp, r, site, nv);
      if (dist_to(E + dE, elo, ehi) <= dist_to(E, elo, ehi)) {
        sp[site] = (int8_t)nv;
        E += dE;
      }
    }
    if (dist_to(E, elo, ehi) == 0) break;
    if (phase == 0) {
      const uint4 r = draw(I, wa++, (uint32_t)loc, kTagWarm);
      const bool below = (W.lo + W.hi) < (I.nbins - 1);
      int a, b;
      if (I.model == kIsing) {
        a = (r.x >> 31) ? 1 : -1;
        b = -a;
      } else {
        a = (int)__umulhi(r.x, (uint32_t)I.q);
        b = a + 1 + (int)__umulhi(r.y, (uint32_t)(I.q - 1));
        b = (b >= I.q) ? b - I.q : b;
      }
      for (int y = 0; y < I.L; ++y)
        for (int x = 0; x < I.L; ++x)
          sp[y * I.L + x] = (int8_t)((below || ((x + y) & 1) == 0) ? a : b);
      E = full_energy(I, sp);
    }
  }
  P.cfg[g] = g;
  P.E[g] = E;
  P.att[g] = 0;
  P.watt[g] = wa;
  if (dist_to(E, elo, ehi) != 0) atomicMin(&P.ist[I.inst].error, -7);
}

// ---------------------------------------------------------------------------
// Flatness and in-window merge: one 256-thread block per window.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_merge_windows(DevPtrs P) {
  __shared__ uint64_t red64[8];
  const int gw = blockIdx.x;
  const WinDesc W = P.win[gw];
  const InstDesc& I = P.inst[W.inst];
  const WinState ws0 = P.wst[gw];
  if (P.ist[W.inst].done || P.ist[W.inst].error || ws0.frozen) return;
  const int m = I.m, nb = W.nb;
  const int tid = threadIdx.x;
  uint8_t* U = P.U + W.u_base;

  // visited union; every walker's H is read here at every check, so the
  // 2^31 guard on the histogram counters sits in this loop
  uint64_t cnt = 0;
  for (int j = tid; j < nb; j += blockDim.x) {
    uint8_t u = U[j];
    for (int k = 0; k < m; ++k) {
      const uint32_t h = P.H[W.lng_base + (int64_t)k * nb + j];
      if (h > 0) u = 1;
      if (h >= 0x80000000u) atomicMin(&P.ist[W.inst].error, -5);
    }
    U[j] = u;
    cnt += u;
  }
  cnt = block_reduce(cnt, [](uint64_t a, uint64_t b) { return a + b; }, red64);
  const bool one_t = I.schedule == kOneOverT;
  const bool phase_b = one_t && ws0.phase == 1;
  bool ready = cnt > 0;
  for (int k = 0; k < m && ready && !phase_b; ++k) {
    uint64_t mn = UINT64_MAX, sm = 0;
    for (int j = tid; j < nb; j += blockDim.x) {
      const uint64_t h = P.H[W.lng_base + (int64_t)k * nb + j];
      sm += h;
      if (U[j] && h < mn) mn = h;
    }
    mn = block_reduce(mn, [](uint64_t a, uint64_t b) { return a < b ? a : b; }, red64);
    sm = block_reduce(sm, [](uint64_t a, uint64_t b) { return a + b; }, red64);
    if (one_t) {
      if (mn == 0) ready = false;
    } else if ((uint64_t)I.flat_den * cnt * mn < (uint64_t)I.flat_num * sm) {
      ready = false;
    }
  }
  if (!ready) return;

  // new ln f: halve (phase A / halving schedule), or 1/t with t the attempts
  // per walker over the visited bins; phase A hands over to B once halving
  // would reach 1/t
  const int slot0 = I.slot_base + (gw - I.win_base) * m;
  const double tinv = (double)cnt / (double)P.att[slot0];
  double next = phase_b ? tinv : 0.5 * ws0.lnf;
  const bool to_b = one_t && !phase_b && next <= tinv;
  if (to_b) next = tinv;
  const bool freezing = next <= I.lnf_final;

  for (int j = tid; j < nb; j += blockDim.x) {
    if (P.prec == kFP64) {
      double v[kMaxWalkersPerWindow];
      for (int k = 0; k < m; ++k) v[k] = P.lng[W.lng_base + (int64_t)k * nb + j];
      if (freezing)
        for (int k = 0; k < m; ++k) P.pieces[W.lng_base + (int64_t)k * nb + j] = v[k];
      int n = m;
      while (n > 1) {
        int o = 0;
        for (int i = 0; i + 1 < n; i += 2) v[o++] = v[i] + v[i + 1];
        if (n & 1) v[o++] = v[n - 1];
        n = o;
      }
      const double mean = v[0] / (double)m;
      if (!isfinite(mean)) atomicMin(&P.ist[W.inst].error, -4);
      for (int k = 0; k < m; ++k) P.lng[W.lng_base + (int64_t)k * nb + j] = mean;
    } else {
      float vh[kMaxWalkersPerWindow], vl[kMaxWalkersPerWindow];
      for (int k = 0; k < m; ++k) {
        vh[k] = P.lhi[W.lng_base + (int64_t)k * nb + j];
        vl[k] = P.llo[W.lng_base + (int64_t)k * nb + j];
      }
      if (freezing)
        for (int k = 0; k < m; ++k)
          P.pieces[W.lng_base + (int64_t)k * nb + j] = (double)vh[k] + (double)vl[k];
      int n = m;
      while (n > 1) {
        int o = 0;
        for (int i = 0; i + 1 < n; i += 2) {
          float a, b;
          df_add(vh[i], vl[i], vh[i + 1], vl[i + 1], a, b);
          vh[o] = a;
          vl[o] = b;
          ++o;
        }
        if (n & 1) {
          vh[o] = vh[n - 1];
          vl[o] = vl[n - 1];
          ++o;
        }
        n = o;
      }
      float mh, ml;
      df_div_int(vh[0], vl[0], m, mh, ml);
      if (!isfinite(mh) || !isfinite(ml)) atomicMin(&P.ist[W.inst].error, -4);
      for (int k = 0; k < m; ++k) {
        P.lhi[W.lng_base + (int64_t)k * nb + j] = mh;
        P.llo[W.lng_base + (int64_t)k * nb + j] = ml;
      }
    }
    for (int k = 0; k < m; ++k) P.H[W.lng_base + (int64_t)k * nb + j] = 0;
  }
  if (tid == 0) {
    WinState ws = ws0;
    if (!phase_b) {
      if (ws.stage < kMaxStages) P.stage_merge[(int64_t)gw * kMaxStages + ws.stage] = P.ist[W.inst].merges;
      ws.stage += 1;
    }
    ws.lnf = next;
    if (to_b) ws.phase = 1;
    if (freezing) ws.frozen = 1;
    P.wst[gw] = ws;
  }
}

__global__ void k_merge_finish(DevPtrs P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n_inst) return;
  InstState st = P.ist[i];
  if (st.done || st.error) return;
  const InstDesc& I = P.inst[i];
  int all = 1;
  for (int w = 0; w < I.h; ++w) all &= P.wst[I.win_base + w].frozen;
  if (all) {
    st.done = 1;
    st.done_merge = st.merges;
  }
  st.merges += 1;
  P.ist[i] = st;
}

// ---------------------------------------------------------------------------
// Replica exchange round: one 64-thread block per lower window w of a pair.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_exchange(DevPtrs P) {
  __shared__ int pi[kMaxWalkersPerWindow];
  __shared__ uint64_t red[1];
  const int gw = blockIdx.x;
  const WinDesc W = P.win[gw];
  const InstDesc& I = P.inst[W.inst];
  const InstState st = P.ist[W.inst];
  if (st.done || st.error) return;
  const int w = gw - I.win_base;
  const uint64_t t = st.rounds;
  if ((uint64_t)(w & 1) != (t & 1) || w + 1 >= I.h) return;
  const int m = I.m;
  const int tid = threadIdx.x;
  if (tid == 0) {
    for (int k = 0; k < m; ++k) pi[k] = k;
    uint4 r = make_uint4(0, 0, 0, 0);
    int used = 4, call = 0;
    for (int i = m - 1; i >= 1; --i) {
      if (used == 4) {
        r = draw(I, t, ((uint32_t)w << 8) | (uint32_t)call++, kTagPerm);
        used = 0;
      }
      const uint32_t rv = used == 0 ? r.x : used == 1 ? r.y : used == 2 ? r.z : r.w;
      ++used;
      const int j = (int)__umulhi(rv, (uint32_t)(i + 1));
      const int tmp = pi[i];
      pi[i] = pi[j];
      pi[j] = tmp;
    }
  }
  __syncthreads();
  const WinDesc Wn = P.win[gw + 1];
  uint64_t tries = 0, inr = 0, acc = 0;
  if (tid < m) {
    const int li = w * m + tid, lj = (w + 1) * m + pi[tid];
    const int si = I.slot_base + li, sj = I.slot_base + lj;
    const int32_t EX = P.E[si], EY = P.E[sj];
    const int bx = (EX - I.emin) >> I.binw_shift, by = (EY - I.emin) >> I.binw_shift;
    tries = 1;
    if (!(by < W.lo || by > W.hi || bx < Wn.lo || bx > Wn.hi)) {
      inr = 1;
      const int64_t bi = W.lng_base + (int64_t)tid * W.nb;
      const int64_t bj = Wn.lng_base + (int64_t)pi[tid] * Wn.nb;
      const int ix = bx - W.lo, iy = by - W.lo, jx = bx - Wn.lo, jy = by - Wn.lo;
      const uint4 r = draw(I, t, (uint32_t)li, kTagAcc);
      bool a;
      if (P.prec == kFP64) {
        const double lnP = (P.lng[bi + ix] - P.lng[bi + iy]) + (P.lng[bj + jy] - P.lng[bj + jx]);
        a = accept64(u53(r.z, r.w), lnP);
      } else {
        const float x1 = (P.lhi[bi + ix] - P.lhi[bi + iy]) + (P.llo[bi + ix] - P.llo[bi + iy]);
        const float x2 = (P.lhi[bj + jy] - P.lhi[bj + jx]) + (P.llo[bj + jy] - P.llo[bj + jx]);
        a = accept32(r.z >> 8, x1 + x2);
      }
      if (a) {
        acc = 1;
        const int32_t ci = P.cfg[si];
        P.cfg[si] = P.cfg[sj];
        P.cfg[sj] = ci;
        P.E[si] = EY;
        P.E[sj] = EX;
      }
    }
  }
  tries = wave_reduce(tries, [](uint64_t a, uint64_t b) { return a + b; });
  inr = wave_reduce(inr, [](uint64_t a, uint64_t b) { return a + b; });
  acc = wave_reduce(acc, [](uint64_t a, uint64_t b) { return a + b; });
  if (tid == 0) {
    P.xstats[3 * gw + 0] += tries;
    P.xstats[3 * gw + 1] += inr;
    P.xstats[3 * gw + 2] += acc;
  }
  (void)red;
}

__global__ void k_exchange_finish(DevPtrs P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P.n_inst) return;
  if (!P.ist[i].done && !P.ist[i].error) P.ist[i].rounds += 1;
}

// ---------------------------------------------------------------------------
// Joining (Sec. 3, Eq. 2) and normalisation, FP64, one block per call.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double beta5(const double* l, int j) {
  return (((l[j - 2] - 8.0 * l[j - 1]) + 8.0 * l[j + 1]) - l[j + 2]) / 12.0;
}

// Joins the window representatives into R (Sec. 3, Eq. 2): the
// first window as it is, then window w from the bin of (w-1, w) where the
// five-point slopes agree best (lowest such bin on ties; the middle of the
// overlap if no bin qualifies), shifted to continue the joined curve.
// normalise: Ising sum g = 2^N, Potts g(E_min) = q.  Whole block.
// rep: this instance's representatives, window w at rep + (rep_off -
// the instance's rep_base).
__device__ void stitch_normalise(const DevPtrs& P, const InstDesc& I, const double* rep, double* R,
                                 int normalise, double* redd, int64_t* redi, double& shift_s,
                                 int& best_s, bool record_joins) {
  const int tid = threadIdx.x, nt = blockDim.x;
  __syncthreads();
  for (int b = tid; b < I.nbins; b += nt) R[b] = -INFINITY;
  __syncthreads();
  {
    const WinDesc W0 = P.win[I.win_base];
    const uint8_t* U0 = P.U + W0.u_base;
    const double* r0 = rep + (W0.rep_off - I.rep_base);
    for (int j = tid; j < W0.nb; j += nt) R[W0.lo + j] = U0[j] ? r0[j] : -INFINITY;
  }
  if (tid == 0) shift_s = 0.0;
  __syncthreads();
  for (int w = 1; w < I.h; ++w) {
    const WinDesc Wa = P.win[I.win_base + w - 1];
    const WinDesc Wb = P.win[I.win_base + w];
    const double* la = rep + (Wa.rep_off - I.rep_base);
    const double* lb = rep + (Wb.rep_off - I.rep_base);
    const uint8_t* Ua = P.U + Wa.u_base;
    const uint8_t* Ub = P.U + Wb.u_base;
    double bestd = INFINITY;
    for (int b = Wb.lo + 2 + tid; b <= Wa.hi - 2; b += nt) {
      bool ok = true;
      for (int d = -2; d <= 2 && ok; ++d) ok = Ua[b + d - Wa.lo] && Ub[b + d - Wb.lo];
      if (!ok) continue;
      const double db = fabs(beta5(la, b - Wa.lo) - beta5(lb, b - Wb.lo));
      if (db < bestd) bestd = db;
    }
    bestd = block_reduce(bestd, [](double a, double b) { return a < b ? a : b; }, redd);
    int64_t bi = INT64_MAX;
    if (bestd < INFINITY) {
      for (int b = Wb.lo + 2 + tid; b <= Wa.hi - 2; b += nt) {
        bool ok = true;
        for (int d = -2; d <= 2 && ok; ++d) ok = Ua[b + d - Wa.lo] && Ub[b + d - Wb.lo];
        if (!ok) continue;
        const double db = fabs(beta5(la, b - Wa.lo) - beta5(lb, b - Wb.lo));
        if (db == bestd && b < bi) bi = b;
      }
    }
    bi = block_reduce(bi, [](int64_t a, int64_t b) { return a < b ? a : b; }, redi);
    if (tid == 0) {
      const int best = (bi == INT64_MAX) ? (Wb.lo + Wa.hi) / 2 : (int)bi;
      best_s = best;
      shift_s = (la[best - Wa.lo] + shift_s) - lb[best - Wb.lo];
      if (record_joins) P.joins[I.win_base + w] = best;
    }
    __syncthreads();
    const int best = best_s;
    const double sh = shift_s;
    for (int b = best + tid; b <= Wb.hi; b += nt)
      R[b] = Ub[b - Wb.lo] ? lb[b - Wb.lo] + sh : -INFINITY;
    __syncthreads();
  }
  if (!normalise) return;
  double c;
  if (I.model == kIsing) {
    double mx = -INFINITY;
    for (int b = tid; b < I.nbins; b += nt) mx = fmax(mx, R[b]);
    mx = block_reduce(mx, [](double a, double b) { return a > b ? a : b; }, redd);
    double acc = 0.0;
    for (int b = tid; b < I.nbins; b += nt)
      if (isfinite(R[b])) acc += exp(R[b] - mx);
    acc = block_reduce(acc, [](double a, double b) { return a + b; }, redd);
    c = (double)I.N * log(2.0) - (mx + log(acc));
  } else {
    c = log((double)I.q) - R[0];
  }
  __syncthreads();
  for (int b = tid; b < I.nbins; b += nt)
    if (isfinite(R[b])) R[b] += c;
}

__global__ __launch_bounds__(256) void k_join(DevPtrs P, int32_t instance, int32_t normalise) {
  __shared__ double redd[8];
  __shared__ int64_t redi[8];
  __shared__ double shift_s;
  __shared__ int best_s;
  const InstDesc& I = P.inst[instance];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = I.m;
  double* R = P.R + I.r_base;
  // window representatives: mean over walkers, same tree as the merge
  for (int w = 0; w < I.h; ++w) {
    const WinDesc W = P.win[I.win_base + w];
    double* rep = P.rep + W.rep_off;
    for (int j = tid; j < W.nb; j += nt) {
      if (P.prec == kFP64) {
        double v[kMaxWalkersPerWindow];
        for (int k = 0; k < m; ++k) v[k] = P.lng[W.lng_base + (int64_t)k * W.nb + j];
        int n = m;
        while (n > 1) {
          int o = 0;
          for (int i = 0; i + 1 < n; i += 2) v[o++] = v[i] + v[i + 1];
          if (n & 1) v[o++] = v[n - 1];
          n = o;
        }
        rep[j] = v[0] / (double)m;
      } else {
        float vh[kMaxWalkersPerWindow], vl[kMaxWalkersPerWindow];
        for (int k = 0; k < m; ++k) {
          vh[k] = P.lhi[W.lng_base + (int64_t)k * W.nb + j];
          vl[k] = P.llo[W.lng_base + (int64_t)k * W.nb + j];
        }
        int n = m;
        while (n > 1) {
          int o = 0;
          for (int i = 0; i + 1 < n; i += 2) {
            float a, b;
            df_add(vh[i], vl[i], vh[i + 1], vl[i + 1], a, b);
            vh[o] = a;
            vl[o] = b;
            ++o;
          }
          if (n & 1) {
            vh[o] = vh[n - 1];
            vl[o] = vl[n - 1];
            ++o;
          }
          n = o;
        }
        float mh, ml;
        df_div_int(vh[0], vl[0], m, mh, ml);
        rep[j] = (double)mh + (double)ml;
      }
    }
  }
  stitch_normalise(P, I, P.rep + I.rep_base, R, normalise, redd, redi, shift_s, best_s, true);
}

// Jackknife over the m pieces per window (Sec. 3): for k = 0..m-1 the
// representatives are the pairwise means of the pieces without walker k,
// joined and normalised into row k of jk; then per bin the mean of the m
// rows and sqrt((m-1)/m * sum (R_k - mean)^2) go to rows m and m + 1 (-inf
// and 0 where any row is not finite).  rep holds the instance's window
// representatives (sum of its window sizes), jk (m + 2) x nbins doubles;
// every element of both is written before it is read.  One block.
__global__ __launch_bounds__(256) void k_jackknife(DevPtrs P, int32_t instance, double* rep_buf,
                                                   double* jk) {
  __shared__ double redd[8];
  __shared__ int64_t redi[8];
  __shared__ double shift_s;
  __shared__ int best_s;
  const InstDesc& I = P.inst[instance];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int m = I.m, nbins = I.nbins;
  for (int k = 0; k < m; ++k) {
    for (int w = 0; w < I.h; ++w) {
      const WinDesc W = P.win[I.win_base + w];
      double* rep = rep_buf + (W.rep_off - I.rep_base);
      for (int j = tid; j < W.nb; j += nt) {
        double v[kMaxWalkersPerWindow];
        int n = 0;
        for (int i = 0; i < m; ++i)
          if (i != k) v[n++] = P.pieces[W.lng_base + (int64_t)i * W.nb + j];
        const int cnt = n;
        while (n > 1) {
          int o = 0;
          for (int i = 0; i + 1 < n; i += 2) v[o++] = v[i] + v[i + 1];
          if (n & 1) v[o++] = v[n - 1];
          n = o;
        }
        rep[j] = v[0] / (double)cnt;
      }
    }
    __syncthreads();
    stitch_normalise(P, I, rep_buf, jk + (int64_t)k * nbins, 1, redd, redi, shift_s, best_s, false);
    __syncthreads();
  }
  for (int b = tid; b < nbins; b += nt) {
    bool fin = true;
    double acc = 0.0;
    for (int k = 0; k < m; ++k) {
      const double r = jk[(int64_t)k * nbins + b];
      fin = fin && isfinite(r);
      acc += r;
    }
    double mu = -INFINITY, e = 0.0;
    if (fin) {
      mu = acc / (double)m;
      double v = 0.0;
      for (int k = 0; k < m; ++k) {
        const double d = jk[(int64_t)k * nbins + b] - mu;
        v += d * d;
      }
      e = sqrt((double)(m - 1) / (double)m * v);
    }
    jk[(int64_t)m * nbins + b] = mu;
    jk[(int64_t)(m + 1) * nbins + b] = e;
  }
}

// Device memory of the allocation-free jackknife (rewl_jackknife_noalloc):
// the window representatives and leave-one-out rows of one instance.  Every
// GPU the library runs on holds its own copy until the process ends; calls
// that overlap on one GPU share it.
static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t scratch_address(double** out) {
  static std::mutex mu;
  static double* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<double*>(p);
  }
  *out = addr[dev];
  return hipSuccess;
}

// Canonical <E> and C_V (Sec. 5, Eqs. 7-8) from the joined ln g: one thread per T.
__global__ void k_thermo(DevPtrs P, int32_t instance, int32_t nT) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nT) return;
  const InstDesc& I = P.inst[instance];
  const double* lng = P.R + I.r_base;
  const double t = P.thermo[i];
  double mx = -INFINITY;
  for (int b = 0; b < I.nbins; ++b) {
    if (!isfinite(lng[b])) continue;
    const double a = lng[b] - (double)(I.emin + b * I.binw) / t;
    if (a > mx) mx = a;
  }
  double z = 0.0, e1 = 0.0;
  for (int b = 0; b < I.nbins; ++b) {
    if (!isfinite(lng[b])) continue;
    const double E = (double)(I.emin + b * I.binw);
    const double wgt = exp(lng[b] - E / t - mx);
    z += wgt;
    e1 += wgt * E;
  }
  const double em = e1 / z;
  double v = 0.0;
  for (int b = 0; b < I.nbins; ++b) {
    if (!isfinite(lng[b])) continue;
    const double E = (double)(I.emin + b * I.binw);
    const double wgt = exp(lng[b] - E / t - mx);
    v += wgt * (E - em) * (E - em);
  }
  P.thermo[kMaxTemps + i] = em;
  P.thermo[2 * kMaxTemps + i] = (v / z) / (t * t);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_init(const DevPtrs& P, hipStream_t s) {
  const int bs = 64;
  hipLaunchKernelGGL(k_init, dim3((P.n_slots + bs - 1) / bs), dim3(bs), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_merge(const DevPtrs& P, hipStream_t s) {
  hipLaunchKernelGGL(k_merge_windows, dim3(P.n_win), dim3(256), 0, s, P);
  hipLaunchKernelGGL(k_merge_finish, dim3((P.n_inst + 63) / 64), dim3(64), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_exchange(const DevPtrs& P, hipStream_t s) {
  hipLaunchKernelGGL(k_exchange, dim3(P.n_win), dim3(64), 0, s, P);
  hipLaunchKernelGGL(k_exchange_finish, dim3((P.n_inst + 63) / 64), dim3(64), 0, s, P);
  return hipGetLastError();
}

hipError_t launch_join(const DevPtrs& P, int32_t instance, int32_t normalise, hipStream_t s) {
  hipLaunchKernelGGL(k_join, dim3(1), dim3(256), 0, s, P, instance, normalise);
  return hipGetLastError();
}

hipError_t launch_jackknife(const DevPtrs& P, int32_t instance, double* rep, double* jk,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_jackknife, dim3(1), dim3(256), 0, s, P, instance, rep, jk);
  return hipGetLastError();
}

hipError_t launch_thermo(const DevPtrs& P, int32_t instance, int32_t nT, hipStream_t s) {
  hipLaunchKernelGGL(k_thermo, dim3((nT + 63) / 64), dim3(64), 0, s, P, instance, nT);
  return hipGetLastError();
}

}  // namespace rewl
