// Host side of librewl: the C-ABI declared in include/rewl.h.
//
// The host validates parameters, derives bins and windows, lays the whole
// simulation state out in the caller's device workspace, builds the
// walker-to-workgroup table for the sweep kernel and enqueues kernels on the
// caller's stream.  It never allocates device memory.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/rewl.h"
#include "rewl_internal.h"

using namespace rewl;

namespace {

constexpr uint64_t kCkptMagic = 0x3330304c5745524bULL;  // "KREWL003"
constexpr size_t kAlign = 256;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Layout {
  std::vector<InstDesc> inst;
  std::vector<WinDesc> win;
  int32_t n_slots = 0;
  int64_t spin_bytes = 0;
  int64_t lng_elems = 0;
  int32_t u_elems = 0;
  int32_t rep_elems = 0;
  int32_t r_elems = 0;
  // per sweep class (Ising L <= 32, Ising L <= 64, Potts): largest lattice
  // in the sweep's LDS format (32-bit words), largest window (bins), whether
  // a q >= 3 Potts instance is present, walkers
  int32_t lat_words[3] = {0, 0, 0};      // with Potts spins as bytes
  int32_t lat_words_nib[3] = {0, 0, 0};  // with Potts spins as nibbles
  int32_t nib_ok[3] = {1, 1, 1};         // every Potts instance has q <= 16
  int32_t nb_max[3] = {0, 0, 0};
  int32_t potts3[3] = {0, 0, 0};
  int32_t walkers[3] = {0, 0, 0};
  int32_t n_max[3] = {0, 0, 0};          // most sites of an instance
  int32_t prec = 0;
  // byte offsets inside the workspace
  int64_t jk_elems = 0;  // largest (m + 2) * nbins of any instance
  size_t o_inst, o_win, o_wg, o_ist, o_wst, o_sm, o_xs, o_cfg, o_E, o_att, o_watt, o_spins,
      o_lng, o_lhi, o_llo, o_H, o_pieces, o_U, o_rep, o_R, o_thermo, o_joins, o_jk, total;
};

// Equal-size windows with overlap num/den over bins 0..nbins-1 (Fig. 1a):
// width W = S/(1+(h-1)(1-o)), lo_i = round(i(1-o)W), hi_i = round((i(1-o)+1)W),
// half rounded up; computed in integers.
void equal_windows(int32_t nbins, int32_t h, int32_t on, int32_t od, int32_t* lo, int32_t* hi) {
  const int64_t S = nbins - 1, d = od - on, D = od + (int64_t)(h - 1) * d;
  for (int i = 0; i < h; ++i) {
    lo[i] = (int32_t)((2 * i * d * S + D) / (2 * D));
    hi[i] = (int32_t)((2 * (i * d + od) * S + D) / (2 * D));
  }
}

int check_params(const rewl_params& p) {
  if (p.model != REWL_ISING && p.model != REWL_POTTS) return REWL_E_INVAL;
  if (p.L < 2 || p.L > kMaxL) return REWL_E_INVAL;
  if (p.model == REWL_POTTS && (p.q < 2 || p.q > 127)) return REWL_E_INVAL;
  if (p.n_windows < 1 || p.walkers_per_window < 1 || p.walkers_per_window > kMaxWalkersPerWindow)
    return REWL_E_INVAL;
  if (p.flat_den <= 0 || p.flat_num < 0 || p.flat_num > p.flat_den) return REWL_E_INVAL;
  if (p.precision != REWL_FP64 && p.precision != REWL_FP32C) return REWL_E_INVAL;
  if (!(p.lnf_init > 0.0) || !(p.lnf_final > 0.0) || !isfinite(p.lnf_init)) return REWL_E_INVAL;
  if (p.overlap_den <= 0 || p.overlap_num < 0 || p.overlap_num >= p.overlap_den) return REWL_E_INVAL;
  if (p.schedule != REWL_HALVING && p.schedule != REWL_ONE_OVER_T) return REWL_E_INVAL;
  if (p.reserved != 0) return REWL_E_INVAL;
  return REWL_OK;
}

int lds_budget_bytes() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
    return v;
  return 160 * 1024;  // gfx950
}

int build_layout(const rewl_params* params, int32_t n, const int32_t* wlo, const int32_t* whi,
                 int lds_budget, Layout& Lo) {
  if (!params || n < 1) return REWL_E_INVAL;
  if ((wlo == nullptr) != (whi == nullptr)) return REWL_E_INVAL;
  Lo = Layout();
  Lo.prec = params[0].precision;
  int32_t slot = 0, win = 0, woff = 0, rep = 0, rbase = 0;
  int64_t spin = 0, lng = 0;
  for (int i = 0; i < n; ++i) {
    const rewl_params& p = params[i];
    int rc = check_params(p);
    if (rc) return rc;
    if (p.precision != Lo.prec) return REWL_E_INVAL;
    InstDesc I{};
    I.model = p.model;
    I.L = p.L;
    I.N = p.L * p.L;
    I.q = p.model == REWL_POTTS ? p.q : 2;
    I.binw = p.model == REWL_ISING ? 4 : (I.q == 2 ? 2 : 1);
    I.binw_shift = I.binw == 4 ? 2 : (I.binw == 2 ? 1 : 0);
    I.emin = -2 * I.N;
    const int32_t emax = p.model == REWL_ISING ? 2 * I.N : 0;
    I.nbins = (emax - I.emin) / I.binw + 1;
    I.h = p.n_windows;
    I.m = p.walkers_per_window;
    I.W = I.h * I.m;
    I.inst = i;
    I.slot_base = slot;
    I.win_base = win;
    I.flat_num = p.flat_num;
    I.flat_den = p.flat_den;
    I.npad = (int32_t)align_up((size_t)I.N, 16);
    I.spin_base = spin;
    I.lnf_final = p.lnf_final;
    I.key0 = (uint32_t)p.seed;
    I.key1 = (uint32_t)(p.seed >> 32);
    I.schedule = p.schedule;
    I.r_base = rbase;
    I.rep_base = rep;
    std::vector<int32_t> lo(I.h), hi(I.h);
    if (wlo) {
      memcpy(lo.data(), wlo + woff, sizeof(int32_t) * I.h);
      memcpy(hi.data(), whi + woff, sizeof(int32_t) * I.h);
      woff += I.h;
    } else {
      equal_windows(I.nbins, I.h, p.overlap_num, p.overlap_den, lo.data(), hi.data());
    }
    I.nbmax = 0;
    for (int w = 0; w < I.h; ++w) {
      if (lo[w] < 0 || hi[w] >= I.nbins || hi[w] - lo[w] < 4) return REWL_E_INVAL;
      if (w > 0 && (lo[w] <= lo[w - 1] || hi[w] <= hi[w - 1] || lo[w] > hi[w - 1])) return REWL_E_INVAL;
      WinDesc D{};
      D.lo = lo[w];
      D.hi = hi[w];
      D.nb = hi[w] - lo[w] + 1;
      D.inst = i;
      D.lng_base = lng;
      D.u_base = Lo.u_elems;
      D.rep_off = rep;
      lng += (int64_t)D.nb * I.m;
      Lo.u_elems += D.nb;
      rep += D.nb;
      I.nbmax = std::max(I.nbmax, D.nb);
      Lo.win.push_back(D);
    }
    const int cls = I.model == REWL_POTTS ? 2 : (I.L <= 32 ? 0 : 1);
    // sweep LDS lattice words: Ising bit rows (1 word per row for L <= 32,
    // else 2), Potts bytes or nibbles
    int lw = I.model == REWL_ISING ? I.L * (I.L <= 32 ? 1 : 2) : (I.N + 3) / 4;
    int lwn = I.model == REWL_ISING ? lw : (I.N + 7) / 8;
    lw += lw & 1;
    lwn += lwn & 1;
    Lo.lat_words[cls] = std::max(Lo.lat_words[cls], lw);
    Lo.lat_words_nib[cls] = std::max(Lo.lat_words_nib[cls], lwn);
    if (I.model == REWL_POTTS && I.q > 16) Lo.nib_ok[cls] = 0;
    Lo.nb_max[cls] = std::max(Lo.nb_max[cls], I.nbmax);
    Lo.potts3[cls] |= (I.model == REWL_POTTS && I.q >= 3);
    Lo.walkers[cls] += I.W;
    Lo.n_max[cls] = std::max(Lo.n_max[cls], I.N);
    slot += I.W;
    win += I.h;
    spin += (int64_t)I.W * I.npad;
    rbase += I.nbins;
    Lo.jk_elems = std::max(Lo.jk_elems, (int64_t)(I.m + 2) * I.nbins);
    Lo.inst.push_back(I);
  }
  Lo.n_slots = slot;
  Lo.spin_bytes = spin;
  Lo.lng_elems = lng;
  Lo.rep_elems = rep;
  Lo.r_elems = rbase;
  // workspace offsets
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, kAlign);
    return at;
  };
  const size_t nw = Lo.win.size();
  Lo.o_inst = take(sizeof(InstDesc) * Lo.inst.size());
  Lo.o_win = take(sizeof(WinDesc) * nw);
  Lo.o_wg = take(sizeof(WgDesc) * (size_t)slot);  // room for one walker per workgroup
  Lo.o_ist = take(sizeof(InstState) * Lo.inst.size());
  Lo.o_wst = take(sizeof(WinState) * nw);
  Lo.o_sm = take(sizeof(int64_t) * kMaxStages * nw);
  Lo.o_xs = take(sizeof(uint64_t) * 3 * nw);
  Lo.o_cfg = take(sizeof(int32_t) * slot);
  Lo.o_E = take(sizeof(int32_t) * slot);
  Lo.o_att = take(sizeof(uint64_t) * slot);
  Lo.o_watt = take(sizeof(uint64_t) * slot);
  Lo.o_spins = take((size_t)spin);
  if (Lo.prec == REWL_FP64) {
    Lo.o_lng = take(sizeof(double) * lng);
    Lo.o_lhi = Lo.o_llo = 0;
  } else {
    Lo.o_lng = 0;
    Lo.o_lhi = take(sizeof(float) * lng);
    Lo.o_llo = take(sizeof(float) * lng);
  }
  Lo.o_H = take(sizeof(uint32_t) * lng);
  Lo.o_pieces = take(sizeof(double) * lng);
  Lo.o_U = take((size_t)Lo.u_elems);
  Lo.o_rep = take(sizeof(double) * rep);
  Lo.o_R = take(sizeof(double) * rbase);
  Lo.o_thermo = take(sizeof(double) * 3 * kMaxTemps);
  Lo.o_joins = take(sizeof(int32_t) * nw);
  Lo.o_jk = take(sizeof(double) * (size_t)Lo.jk_elems);
  Lo.total = o;
  return REWL_OK;
}

// Sweep launch plan, per kernel class: walkers per workgroup (G, one
// wavefront), ln g page slots (P, a power of two), LDS bytes and the class's
// slice of the workgroup table.  Per lane a class needs 4 * lat_words +
// 12 * P bytes of LDS.  The page must hold bin +- 2D (D = 4 for q >= 3
// Potts, else 2), so P >= 32 or 16, unless the largest window fits whole
// (P = the power of two that holds it).  By default P is the largest page
// that still lets T = 4 (else 3, 2, 1) full workgroups share a compute unit.
struct ClassPlan {
  int32_t G = 0, P = 0, count = 0, offset = 0;
  int32_t prod = 0;  // RNG producer wavefront per workgroup
  int32_t nib = 0;   // Potts spins: 0 bytes, 1 nibbles with the neighbour table, 2 nibbles
  size_t lds_bytes = 0;
};
// Batch-level choices: fused = every class in one launch (one LDS size, one
// RNG-producer setting) rather than one launch per class on forked streams;
// splits = launches a sweep of F attempts is cut into (same results, the
// workgroups are placed afresh for each part); order = order of the
// workgroup table for a fused launch (0 by class, 1 classes reversed,
// 2 classes interleaved), i.e. which workgroups the hardware starts first.
struct LaunchPlan {
  ClassPlan cls[3];
  int32_t fused = 0, splits = 1, order = 0;
  std::vector<WgDesc> wg;
};

int class_of(const InstDesc& I) { return I.model == REWL_POTTS ? 2 : (I.L <= 32 ? 0 : 1); }

int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// Smallest and largest useful page of a class.
void page_range(const Layout& Lo, int cls, int& pmin, int& pmax) {
  pmax = pow2_ceil(Lo.nb_max[cls]);
  pmin = std::min(Lo.potts3[cls] ? 32 : 16, pmax);
}

// LDS bytes of a workgroup of G walkers with page P: lattices and pages,
// then (tab bytes, 8-byte aligned) the neighbour table of nibble Potts
// lattices, then with a producer the RNG double buffer (16-byte aligned)
// and a flag word.
size_t lds_of(int lat, int G, int P, int prod, size_t tab) {
  const size_t tab_end = (tab ? align_up((size_t)G * (lat + 12 * P), 8) : (size_t)G * (lat + 12 * P)) + tab;
  return prod ? align_up(tab_end, 16) + (size_t)2 * kRngChunk * G * 16 + 16 : tab_end;
}

// Neighbour-table bytes of a class (8 per site of its largest lattice),
// kept with nibble Potts lattices in form 1.
size_t tab_of(const Layout& Lo, int cls, int nib) { return cls == 2 && nib == 1 ? (size_t)8 * Lo.n_max[cls] : 0; }

int n_compute_units() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
    return v;
  return 256;  // MI355X
}

int plan_class(const Layout& Lo, int cls, int lds_budget, int page_req, int g_req, int prod_req,
               int nib_req, ClassPlan& cp) {
  cp = ClassPlan();
  if (Lo.walkers[cls] == 0) return REWL_OK;
  // Potts nibbles halve the lattice and so raise the workgroups per compute
  // unit, at a little extra latency per attempt: by default when the class
  // has more workgroups than the GPU has compute units
  const bool many = (Lo.walkers[cls] + kSweepWave - 1) / kSweepWave > n_compute_units();
  int nib = cls == 2 && Lo.nib_ok[cls] ? (nib_req < 0 ? (many ? 1 : 0) : nib_req) : 0;
  if (nib_req >= 1 && !(cls == 2 && Lo.nib_ok[cls])) nib = 0;
  const int lat = 4 * (nib ? Lo.lat_words_nib[cls] : Lo.lat_words[cls]);
  const size_t tab = tab_of(Lo, cls, nib);
  int pmin, pmax;
  page_range(Lo, cls, pmin, pmax);
  int P = 0, G = kSweepWave;
  if (page_req > 0) {
    P = std::min(std::max(pow2_ceil(page_req), pmin), pmax);
  } else {
    for (int T = 4; T >= 1 && P == 0; --T) {
      for (int p = pmax; p >= pmin; p >>= 1) {
        if ((size_t)T * lds_of(lat, kSweepWave, p, 0, tab) <= (size_t)lds_budget) {
          P = p;
          break;
        }
      }
    }
    if (P == 0) P = pmin;
  }
  if (g_req > 0) G = std::min(g_req, kSweepWave);
  // producer by default when the class's workgroups do not outnumber the
  // compute units (the walkers' chain, not issue, then bounds the sweep)
  int prod = prod_req;
  if (prod < 0) prod = (Lo.walkers[cls] + G - 1) / G <= n_compute_units() ? 1 : 0;
  while (G > 1 && lds_of(lat, G, P, prod, tab) > (size_t)lds_budget) --G;
  if (lds_of(lat, G, P, prod, tab) > (size_t)lds_budget) return REWL_E_INVAL;
  cp.G = G;
  cp.P = P;
  cp.prod = prod;
  cp.nib = nib;
  cp.lds_bytes = lds_of(lat, G, P, prod, tab);
  return REWL_OK;
}

// Builds the workgroup table: runs of up to G consecutive walkers of one
// instance, class 0 first, then 1, then 2 (each class contiguous, as the
// per-class launches need).  A fused plan may reorder the table: classes
// reversed, or interleaved one workgroup of each class at a time.
void fill_table(const Layout& Lo, LaunchPlan& pl) {
  std::vector<WgDesc> per[3];
  for (int cls = 0; cls < 3; ++cls) {
    const ClassPlan& cp = pl.cls[cls];
    if (cp.G <= 0) continue;
    for (const InstDesc& I : Lo.inst) {
      if (class_of(I) != cls) continue;
      for (int s0 = 0; s0 < I.W; s0 += cp.G) {
        WgDesc d{};
        d.inst = I.inst;
        d.slot_first = I.slot_base + s0;
        d.count = std::min(cp.G, I.W - s0);
        d.cls = cls;
        per[cls].push_back(d);
      }
    }
  }
  pl.wg.clear();
  const int order = pl.fused ? pl.order : 0;
  if (order == 2) {
    size_t at[3] = {0, 0, 0};
    for (bool more = true; more;) {
      more = false;
      for (int cls = 0; cls < 3; ++cls)
        if (at[cls] < per[cls].size()) {
          pl.wg.push_back(per[cls][at[cls]++]);
          more = true;
        }
    }
  } else {
    for (int k = 0; k < 3; ++k) {
      const int cls = order == 1 ? 2 - k : k;
      pl.wg.insert(pl.wg.end(), per[cls].begin(), per[cls].end());
    }
  }
  // per-class slices (meaningful for the per-class launches, order 0)
  for (int cls = 0; cls < 3; ++cls) {
    pl.cls[cls].count = (int32_t)per[cls].size();
    pl.cls[cls].offset = 0;
    for (size_t i = 0; i < pl.wg.size(); ++i)
      if (pl.wg[i].cls == cls) {
        pl.cls[cls].offset = (int32_t)i;
        break;
      }
  }
}

// A fused launch needs one RNG-producer setting for every class present.
bool fusable(const Layout& Lo, const LaunchPlan& pl) {
  int prod = -1, classes = 0;
  for (int cls = 0; cls < 3; ++cls) {
    if (Lo.walkers[cls] == 0) continue;
    ++classes;
    if (prod >= 0 && pl.cls[cls].prod != prod) return false;
    prod = pl.cls[cls].prod;
  }
  return classes > 0;
}

int plan_launch(const Layout& Lo, int lds_budget, int page_req, int g_req, LaunchPlan& pl) {
  pl = LaunchPlan();
  for (int cls = 0; cls < 3; ++cls) {
    int rc = plan_class(Lo, cls, lds_budget, page_req, g_req, -1, -1, pl.cls[cls]);
    if (rc) return rc;
  }
  fill_table(Lo, pl);
  return REWL_OK;
}

}  // namespace

struct rewl_ctx {
  Layout lo;
  LaunchPlan plan;
  std::vector<rewl_params> params;
  std::vector<int32_t> wlo, whi;
  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  // Sweeps of different kernel classes touch disjoint instances and run
  // side by side: class k > first on side[k-1], forked from and joined
  // back to `stream` by events (also inside a captured graph).
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t fork = nullptr;
  hipEvent_t join[2] = {nullptr, nullptr};
  DevPtrs P{};
  hipGraphExec_t graph = nullptr;
  int64_t graph_flips = -1;
  int64_t graph_cycles = 0;
  // the allocation-free jackknife's device array on this context's GPU
  double* scratch = nullptr;
};

namespace {

template <typename T>
T* at(rewl_ctx* c, size_t off) {
  return reinterpret_cast<T*>(c->ws + off);
}

void fill_ptrs(rewl_ctx* c) {
  const Layout& L = c->lo;
  DevPtrs& P = c->P;
  P.inst = at<InstDesc>(c, L.o_inst);
  P.win = at<WinDesc>(c, L.o_win);
  P.wg = at<WgDesc>(c, L.o_wg);
  P.ist = at<InstState>(c, L.o_ist);
  P.wst = at<WinState>(c, L.o_wst);
  P.stage_merge = at<int64_t>(c, L.o_sm);
  P.xstats = at<uint64_t>(c, L.o_xs);
  P.cfg = at<int32_t>(c, L.o_cfg);
  P.E = at<int32_t>(c, L.o_E);
  P.att = at<uint64_t>(c, L.o_att);
  P.watt = at<uint64_t>(c, L.o_watt);
  P.spins = at<int8_t>(c, L.o_spins);
  P.lng = L.prec == REWL_FP64 ? at<double>(c, L.o_lng) : nullptr;
  P.lhi = L.prec == REWL_FP32C ? at<float>(c, L.o_lhi) : nullptr;
  P.llo = L.prec == REWL_FP32C ? at<float>(c, L.o_llo) : nullptr;
  P.H = at<uint32_t>(c, L.o_H);
  P.pieces = at<double>(c, L.o_pieces);
  P.U = at<uint8_t>(c, L.o_U);
  P.rep = at<double>(c, L.o_rep);
  P.R = at<double>(c, L.o_R);
  P.thermo = at<double>(c, L.o_thermo);
  P.joins = at<int32_t>(c, L.o_joins);
  P.jk = at<double>(c, L.o_jk);
  P.n_inst = (int32_t)L.inst.size();
  P.n_win = (int32_t)L.win.size();
  P.n_slots = L.n_slots;
  P.n_wg = (int32_t)c->plan.wg.size();
  P.prec = L.prec;
}

int hip_rc(hipError_t e) { return e == hipSuccess ? REWL_OK : REWL_E_HIP; }

int sync(rewl_ctx* c) { return hip_rc(hipStreamSynchronize(c->stream)); }

template <typename T>
int d2h(rewl_ctx* c, T* dst, const void* src, size_t count) {
  if (!dst || count == 0) return REWL_OK;
  hipError_t e = hipMemcpyAsync(dst, src, sizeof(T) * count, hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return REWL_E_HIP;
  return sync(c);
}

SweepShape shape_of(const rewl_ctx* c, int cls) {
  const ClassPlan& cp = c->plan.cls[cls];
  return SweepShape{cp.G, cp.nib ? c->lo.lat_words_nib[cls] : c->lo.lat_words[cls], cp.P, cp.offset,
                    cp.nib != 0 ? 1 : 0, cls == 2 && cp.nib == 1 ? 1 : 0};
}

// Attempts of part k of a sweep of `flips` cut into `parts` launches.
int64_t part_flips(int64_t flips, int parts, int k) {
  return flips / parts + (k < flips % parts ? 1 : 0);
}

hipError_t enqueue_sweeps(rewl_ctx* c, int64_t flips) {
  const int parts = std::max(1, c->plan.splits);
  hipError_t e = hipSuccess;
  if (c->plan.fused) {
    SweepShape sh[3];
    size_t lds = 0;
    for (int cls = 0; cls < 3; ++cls) {
      sh[cls] = shape_of(c, cls);
      lds = std::max(lds, c->plan.cls[cls].lds_bytes);
    }
    int prod = 0;
    for (int cls = 0; cls < 3; ++cls)
      if (c->plan.cls[cls].count > 0) prod = c->plan.cls[cls].prod;
    for (int k = 0; k < parts && e == hipSuccess; ++k) {
      const int64_t f = part_flips(flips, parts, k);
      if (f > 0) e = launch_sweep_fused(c->P, sh, (int32_t)c->plan.wg.size(), f, lds, prod != 0, c->stream);
    }
    return e;
  }
  int active[3], n = 0;
  for (int cls = 0; cls < 3; ++cls)
    if (c->plan.cls[cls].count > 0) active[n++] = cls;
  const bool fork = n > 1 && c->side[0] != nullptr;
  if (fork) {
    e = hipEventRecord(c->fork, c->stream);
    for (int i = 1; i < n && e == hipSuccess; ++i) e = hipStreamWaitEvent(c->side[i - 1], c->fork, 0);
  }
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    const int cls = active[i];
    const ClassPlan& cp = c->plan.cls[cls];
    const SweepShape sh = shape_of(c, cls);
    hipStream_t s = (fork && i > 0) ? c->side[i - 1] : c->stream;
    for (int k = 0; k < parts && e == hipSuccess; ++k) {
      const int64_t f = part_flips(flips, parts, k);
      if (f > 0) e = launch_sweep_class(c->P, cls, sh, cp.count, f, cp.lds_bytes, cp.prod != 0, s);
    }
  }
  if (fork) {
    for (int i = 1; i < n && e == hipSuccess; ++i) {
      e = hipEventRecord(c->join[i - 1], c->side[i - 1]);
      if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->join[i - 1], 0);
    }
  }
  return e;
}

void destroy_side_streams(rewl_ctx* c) {
  for (int i = 0; i < 2; ++i) {
    if (c->side[i]) (void)hipStreamDestroy(c->side[i]);
    if (c->join[i]) (void)hipEventDestroy(c->join[i]);
    c->side[i] = nullptr;
    c->join[i] = nullptr;
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  c->fork = nullptr;
}

// Side streams for concurrent sweep classes, when the batch has more than one.
hipError_t create_side_streams(rewl_ctx* c) {
  int classes = 0;
  for (int cls = 0; cls < 3; ++cls) classes += c->lo.walkers[cls] > 0;
  if (classes < 2) return hipSuccess;
  hipError_t e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->join[i], hipEventDisableTiming);
  }
  if (e != hipSuccess) destroy_side_streams(c);
  return e;
}

int enqueue_cycle(rewl_ctx* c, int64_t flips) {
  hipError_t e = enqueue_sweeps(c, flips);
  if (e == hipSuccess) e = launch_merge(c->P, c->stream);
  if (e == hipSuccess) e = launch_exchange(c->P, c->stream);
  return hip_rc(e);
}

}  // namespace

extern "C" {

size_t rewl_workspace_bytes(const rewl_params* params, int32_t n, const int32_t* win_lo,
                            const int32_t* win_hi) {
  Layout L;
  if (build_layout(params, n, win_lo, win_hi, lds_budget_bytes(), L) != REWL_OK) return 0;
  return L.total;
}

int rewl_init(const rewl_params* params, int32_t n, const int32_t* win_lo, const int32_t* win_hi,
              void* d_workspace, size_t workspace_bytes, void* stream, rewl_ctx** out) {
  if (!out || !d_workspace) return REWL_E_INVAL;
  *out = nullptr;
  rewl_ctx* c = new (std::nothrow) rewl_ctx();
  if (!c) return REWL_E_NOMEM;
  int rc = build_layout(params, n, win_lo, win_hi, lds_budget_bytes(), c->lo);
  if (!rc) rc = plan_launch(c->lo, lds_budget_bytes(), 0, 0, c->plan);
  if (rc) {
    delete c;
    return rc;
  }
  if (workspace_bytes < c->lo.total) {
    delete c;
    return REWL_E_NOMEM;
  }
  c->params.assign(params, params + n);
  if (win_lo) {
    size_t nw = c->lo.win.size();
    c->wlo.assign(win_lo, win_lo + nw);
    c->whi.assign(win_hi, win_hi + nw);
  }
  c->ws = static_cast<unsigned char*>(d_workspace);
  c->ws_bytes = workspace_bytes;
  c->stream = static_cast<hipStream_t>(stream);
  fill_ptrs(c);
  const Layout& L = c->lo;
  hipError_t e = hipMemsetAsync(c->ws, 0, L.total, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + L.o_inst, L.inst.data(), sizeof(InstDesc) * L.inst.size(),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + L.o_win, L.win.data(), sizeof(WinDesc) * L.win.size(),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + L.o_wg, c->plan.wg.data(), sizeof(WgDesc) * c->plan.wg.size(),
                       hipMemcpyHostToDevice, c->stream);
  std::vector<WinState> ws(L.win.size());
  std::vector<InstState> is(L.inst.size());
  for (size_t i = 0; i < L.inst.size(); ++i) {
    const rewl_params& p = params[i];
    int all = 1;
    for (int w = 0; w < L.inst[i].h; ++w) {
      WinState& s = ws[L.inst[i].win_base + w];
      s.lnf = p.lnf_init;
      s.stage = 0;
      s.frozen = p.lnf_init <= p.lnf_final;
      s.phase = 0;
      s.pad = 0;
      all &= s.frozen;
    }
    is[i].done = all;
    is[i].error = 0;
    is[i].done_merge = -1;
    is[i].merges = 0;
    is[i].rounds = 0;
  }
  std::vector<int64_t> sm((size_t)kMaxStages * L.win.size(), -1);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + L.o_wst, ws.data(), sizeof(WinState) * ws.size(),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + L.o_ist, is.data(), sizeof(InstState) * is.size(),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + L.o_sm, sm.data(), sizeof(int64_t) * sm.size(),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = prepare_sweep_lds((size_t)lds_budget_bytes());
  if (e == hipSuccess) e = scratch_address(&c->scratch);
  if (e == hipSuccess) e = launch_init(c->P, c->stream);
  // host vectors above are pageable; make sure the copies finished
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = create_side_streams(c);
  if (e != hipSuccess) {
    destroy_side_streams(c);
    delete c;
    return REWL_E_HIP;
  }
  *out = c;
  return REWL_OK;
}

int rewl_run_sweeps(rewl_ctx* c, int64_t flips) {
  if (!c || flips < 0) return REWL_E_INVAL;
  if (flips == 0) return REWL_OK;
  return hip_rc(enqueue_sweeps(c, flips));
}

}  // extern "C"

namespace {

// Installs a plan: waits for queued sweeps (they read the old table),
// uploads the workgroup table, drops a captured graph.
int install_plan(rewl_ctx* c, const LaunchPlan& pl) {
  int rc = sync(c);
  if (rc) return rc;
  c->plan = pl;
  fill_ptrs(c);
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  rc = hip_rc(hipMemcpyAsync(c->ws + c->lo.o_wg, c->plan.wg.data(),
                             sizeof(WgDesc) * c->plan.wg.size(), hipMemcpyHostToDevice, c->stream));
  if (!rc) rc = sync(c);
  return rc;
}

void plan_out(const LaunchPlan& pl, int32_t* out) {
  if (!out) return;
  for (int cls = 0; cls < 3; ++cls) {
    out[6 * cls + 0] = pl.cls[cls].P;
    out[6 * cls + 1] = pl.cls[cls].G;
    out[6 * cls + 2] = (int32_t)pl.cls[cls].lds_bytes;
    out[6 * cls + 3] = pl.cls[cls].count;
    out[6 * cls + 4] = pl.cls[cls].prod;
    out[6 * cls + 5] = pl.cls[cls].nib;
  }
  out[18] = pl.fused;
  out[19] = pl.splits;
  out[20] = pl.order;
}

}  // namespace

extern "C" {

int rewl_set_launch(rewl_ctx* c, int32_t cls, int32_t page_bins, int32_t walkers_per_group,
                    int32_t rng_producer, int32_t potts_nibbles, int32_t* out) {
  if (!c || page_bins < 0 || walkers_per_group < 0 || cls < -1 || cls > 2) return REWL_E_INVAL;
  if (rng_producer < -1 || rng_producer > 1 || potts_nibbles < -1 || potts_nibbles > 2)
    return REWL_E_INVAL;
  LaunchPlan pl = c->plan;
  for (int k = 0; k < 3; ++k) {
    if (cls >= 0 && k != cls) continue;
    int rc = plan_class(c->lo, k, lds_budget_bytes(), page_bins, walkers_per_group, rng_producer,
                        potts_nibbles, pl.cls[k]);
    if (rc) return rc;
  }
  // a fused launch needs one producer setting; a class change that breaks
  // it returns the batch to per-class launches
  if (pl.fused && !fusable(c->lo, pl)) pl.fused = 0;
  fill_table(c->lo, pl);
  int rc = install_plan(c, pl);
  if (!rc) plan_out(c->plan, out);
  return rc;
}

int rewl_set_batching(rewl_ctx* c, int32_t fused, int32_t splits, int32_t order, int32_t* out) {
  if (!c || fused < 0 || fused > 1 || splits < 1 || splits > 64 || order < 0 || order > 2)
    return REWL_E_INVAL;
  LaunchPlan pl = c->plan;
  pl.fused = fused;
  pl.splits = splits;
  pl.order = order;
  if (fused && !fusable(c->lo, pl)) return REWL_E_INVAL;
  fill_table(c->lo, pl);
  int rc = install_plan(c, pl);
  if (!rc) plan_out(c->plan, out);
  return rc;
}

int rewl_autotune(rewl_ctx* c, int64_t flips, int32_t repeats, int32_t* out) {
  if (!c || flips <= 0 || repeats < 1) return REWL_E_INVAL;
  const Layout& L = c->lo;
  const int budget = lds_budget_bytes();
  // snapshot the state; every candidate starts from it and it is restored
  // at the end, so tuning does not change the simulation
  std::vector<unsigned char> snap(L.total);
  int rc = d2h(c, snap.data(), c->ws, L.total);
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return REWL_E_HIP;
  // Every timing starts from the snapshot: the same walkers do the same
  // attempts for every candidate (a sweep writes only the state between
  // the instance table and the frozen pieces, so only that is restored).
  // A candidate's time is the median of `repeats` sweeps: the placement of
  // concurrent classes on the compute units varies from sweep to sweep,
  // and a median is not pulled by one unlucky placement.
  const size_t r_lo = L.o_ist, r_hi = L.o_pieces;
  auto time_plan = [&](const LaunchPlan& pl, int reps, bool mean, float& ms) -> int {
    LaunchPlan q = pl;
    fill_table(L, q);
    int r = install_plan(c, q);
    std::vector<float> ts;
    for (int k = 0; k < reps && !r; ++k) {
      r = hip_rc(hipMemcpyAsync(c->ws + r_lo, snap.data() + r_lo, r_hi - r_lo, hipMemcpyHostToDevice,
                                c->stream));
      if (!r) r = hip_rc(hipEventRecord(e0, c->stream));
      if (!r) r = hip_rc(enqueue_sweeps(c, flips));
      if (!r) r = hip_rc(hipEventRecord(e1, c->stream));
      if (!r) r = sync(c);
      float t = 0.0f;
      if (!r) r = hip_rc(hipEventElapsedTime(&t, e0, e1));
      ts.push_back(t);
    }
    if (!r) {
      std::sort(ts.begin(), ts.end());
      const size_t n = ts.size();
      float sum = 0.0f;
      for (float t : ts) sum += t;
      ms = mean ? sum / (float)n : (n % 2 ? ts[n / 2] : 0.5f * (ts[n / 2 - 1] + ts[n / 2]));
    }
    return r;
  };
  // Classes sweep side by side and share the compute units, so every
  // candidate is timed on the whole batch.  The five best plans are kept
  // and decided between at the end (below).
  // The best plan of each form (per-class launches, one fused launch) is
  // kept as well and joins the finalists if the five best lack its form:
  // a per-class plan can reach the top five on lucky placements alone.
  constexpr int kKeep = 5;
  std::vector<std::pair<float, LaunchPlan>> top;
  std::pair<float, LaunchPlan> best_form[2] = {{INFINITY, LaunchPlan()}, {INFINITY, LaunchPlan()}};
  auto consider = [&](const LaunchPlan& pl) -> int {
    float ms = 0.0f;
    const int r = time_plan(pl, repeats, false, ms);
    if (r) return r;
    if (ms < best_form[pl.fused ? 1 : 0].first) best_form[pl.fused ? 1 : 0] = {ms, pl};
    top.emplace_back(ms, pl);
    std::stable_sort(top.begin(), top.end(),
                     [](const std::pair<float, LaunchPlan>& x, const std::pair<float, LaunchPlan>& y) {
                       return x.first < y.first;
                     });
    if ((int)top.size() > kKeep) top.resize(kKeep);
    return REWL_OK;
  };
  auto best = [&]() -> const LaunchPlan& { return top.front().second; };
  rc = consider(c->plan);
  int pmin_all = 1 << 30, pmax_all = 0, classes = 0;
  for (int cls = 0; cls < 3; ++cls) {
    if (L.walkers[cls] == 0) continue;
    int pmin, pmax;
    page_range(L, cls, pmin, pmax);
    pmin_all = std::min(pmin_all, pmin);
    pmax_all = std::max(pmax_all, pmax);
    ++classes;
  }
  // Seeds: one page for every class (clamped to each class's useful
  // range), with and without the RNG producer, Potts spins as nibbles or
  // bytes; per-class launches and, with several classes, the fused launch
  // in each workgroup order.
  for (int p = pmin_all; p <= pmax_all && !rc; p <<= 1)
    for (int prod = 0; prod < 2 && !rc; ++prod)
      for (int nib = 0; nib < (L.walkers[2] > 0 && L.nib_ok[2] ? 3 : 1) && !rc; ++nib) {
        LaunchPlan pl = c->plan;
        pl.fused = 0;
        pl.splits = 1;
        pl.order = 0;
        bool ok = true;
        for (int cls = 0; cls < 3 && ok; ++cls) {
          if (L.walkers[cls] == 0) continue;
          int pmin, pmax;
          page_range(L, cls, pmin, pmax);
          const int pc = std::min(std::max(p, pmin), pmax);
          ok = plan_class(L, cls, budget, pc, 0, prod, cls == 2 ? nib : 0, pl.cls[cls]) == 0;
        }
        if (!ok) continue;
        rc = consider(pl);
        for (int order = 0; order < 3 && classes > 1 && !rc; ++order) {
          pl.fused = 1;
          pl.order = order;
          rc = consider(pl);
        }
      }
  // Then coordinate descent, two passes over the classes: every shape of
  // one class with the others at their best so far (a fused plan stays
  // fused while the producer settings agree).
  for (int step = 0; step < 6 && !rc; ++step) {
    const int cls = step % 3;
    if (L.walkers[cls] == 0) continue;
    int pmin, pmax;
    page_range(L, cls, pmin, pmax);
    const LaunchPlan from = best();
    for (int p = pmin; p <= pmax && !rc; p <<= 1)
      for (int prod = 0; prod < 2 && !rc; ++prod)
        for (int nib = 0; nib < (cls == 2 && L.nib_ok[cls] ? 3 : 1) && !rc; ++nib) {
          LaunchPlan pl = from;
          if (plan_class(L, cls, budget, p, 0, prod, nib, pl.cls[cls])) continue;
          if (pl.fused && !fusable(L, pl)) pl.fused = 0;
          rc = consider(pl);
        }
  }
  // Batch-level choices on the best shapes: the sweep in 2 or 4 launches,
  // and with several classes the other fused orders and per-class launches.
  if (!rc) {
    const LaunchPlan base = best();
    for (int splits : {1, 2, 4}) {
      for (int fused = 0; fused < (classes > 1 ? 2 : 1) && !rc; ++fused) {
        for (int order = 0; order < (fused ? 3 : 1) && !rc; ++order) {
          LaunchPlan pl = base;
          pl.splits = splits;
          pl.fused = fused;
          pl.order = order;
          if (fused && !fusable(L, pl)) continue;
          if (pl.splits == base.splits && pl.fused == base.fused && pl.order == base.order) continue;
          rc = consider(pl);
        }
      }
    }
  }
  // The kept plans decided as a run would use them: `repeats` whole cycles
  // (sweep, merge, exchange) enqueued back to back from the saved state
  // with no host synchronisation between them, an event between cycles;
  // interleaved between the finalists four times; score = mean + standard
  // deviation of the 4 x repeats cycle times.  Per-class launches are placed
  // differently when the host waits after every sweep than when cycles
  // queue up behind each other, and a plan whose time swings with the
  // placement of concurrent kernels pays for its swings.  Merges and
  // exchanges change more than the sweep state, so the whole workspace is
  // restored before every run (and the plan's workgroup table rewritten).
  LaunchPlan chosen = c->plan;
  if (!rc && !top.empty()) {
    std::vector<std::pair<float, LaunchPlan>> finalists = top;
    for (int form = 0; form < 2; ++form) {
      bool present = false;
      for (const auto& f : finalists) present = present || (f.second.fused != 0) == (form == 1);
      if (!present && best_form[form].first < INFINITY) finalists.push_back(best_form[form]);
    }
    std::vector<hipEvent_t> ev((size_t)repeats + 1, nullptr);
    for (auto& x : ev)
      if (!rc) rc = hip_rc(hipEventCreate(&x));
    std::vector<std::vector<float>> times(finalists.size());
    for (int round = 0; round < 4 && !rc; ++round) {
      for (size_t f = 0; f < finalists.size() && !rc; ++f) {
        LaunchPlan q = finalists[f].second;
        fill_table(L, q);
        rc = hip_rc(hipMemcpyAsync(c->ws, snap.data(), L.total, hipMemcpyHostToDevice, c->stream));
        if (!rc) rc = install_plan(c, q);
        if (!rc) rc = hip_rc(hipEventRecord(ev[0], c->stream));
        for (int k = 0; k < repeats && !rc; ++k) {
          rc = enqueue_cycle(c, flips);
          if (!rc) rc = hip_rc(hipEventRecord(ev[k + 1], c->stream));
        }
        if (!rc) rc = sync(c);
        for (int k = 0; k < repeats && !rc; ++k) {
          float t = 0.0f;
          rc = hip_rc(hipEventElapsedTime(&t, ev[k], ev[k + 1]));
          times[f].push_back(t);
        }
      }
    }
    for (auto& x : ev)
      if (x) (void)hipEventDestroy(x);
    float best_score = INFINITY;
    for (size_t f = 0; f < finalists.size() && !rc; ++f) {
      double sum = 0.0, sq = 0.0;
      for (float t : times[f]) sum += t;
      const double mean = sum / (double)times[f].size();
      for (float t : times[f]) sq += ((double)t - mean) * ((double)t - mean);
      const float score = (float)(mean + sqrt(sq / (double)times[f].size()));
      if (score < best_score) {
        best_score = score;
        chosen = finalists[f].second;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // restore the whole saved state, then the chosen plan's workgroup table
  fill_table(L, chosen);
  if (!rc) rc = hip_rc(hipMemcpyAsync(c->ws, snap.data(), L.total, hipMemcpyHostToDevice, c->stream));
  if (!rc) rc = install_plan(c, chosen);
  if (!rc) rc = sync(c);
  if (!rc) plan_out(c->plan, out);
  return rc;
}

int rewl_merge(rewl_ctx* c) {
  if (!c) return REWL_E_INVAL;
  return hip_rc(launch_merge(c->P, c->stream));
}

int rewl_exchange(rewl_ctx* c) {
  if (!c) return REWL_E_INVAL;
  return hip_rc(launch_exchange(c->P, c->stream));
}

int rewl_run_cycles(rewl_ctx* c, int64_t cycles, int64_t flips, int32_t use_graph) {
  if (!c || cycles < 0 || flips < 0) return REWL_E_INVAL;
  if (!use_graph) {
    for (int64_t i = 0; i < cycles; ++i) {
      int rc = enqueue_cycle(c, flips);
      if (rc) return rc;
    }
    return REWL_OK;
  }
  // Capture a batch of cycles once and replay it on the caller's stream.
  // Capture runs on a private stream (the legacy null stream cannot be
  // captured); the captured kernels contain no memset/memcpy nodes.
  const int64_t per_graph = std::min<int64_t>(cycles, 16);
  if (!c->graph || c->graph_flips != flips || c->graph_cycles != per_graph) {
    if (c->graph) {
      (void)hipGraphExecDestroy(c->graph);
      c->graph = nullptr;
    }
    hipStream_t cap = nullptr;
    if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return REWL_E_HIP;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? REWL_OK : REWL_E_HIP;
    hipStream_t user = c->stream;
    c->stream = cap;
    for (int64_t i = 0; i < per_graph && rc == REWL_OK; ++i) rc = enqueue_cycle(c, flips);
    c->stream = user;
    if (e == hipSuccess) e = hipStreamEndCapture(cap, &g);
    (void)hipStreamDestroy(cap);
    if (rc || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return REWL_E_HIP;
    }
    e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->graph = nullptr;
      return REWL_E_HIP;
    }
    c->graph_flips = flips;
    c->graph_cycles = per_graph;
  }
  int64_t done = 0;
  while (done + per_graph <= cycles) {
    if (hipGraphLaunch(c->graph, c->stream) != hipSuccess) return REWL_E_HIP;
    done += per_graph;
  }
  for (; done < cycles; ++done) {
    int rc = enqueue_cycle(c, flips);
    if (rc) return rc;
  }
  return REWL_OK;
}

int rewl_status(rewl_ctx* c, int32_t instance, rewl_instance_status* out, int32_t* stage,
                int32_t* frozen, double* lnf) {
  if (!c || !out || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  const InstDesc& I = c->lo.inst[instance];
  InstState st;
  int rc = d2h(c, &st, c->P.ist + instance, 1);
  if (rc) return rc;
  std::vector<WinState> ws(I.h);
  rc = d2h(c, ws.data(), c->P.wst + I.win_base, (size_t)I.h);
  if (rc) return rc;
  std::vector<uint64_t> att(I.W);
  rc = d2h(c, att.data(), c->P.att + I.slot_base, (size_t)I.W);
  if (rc) return rc;
  out->done = st.done;
  out->error = st.error;
  out->done_merge = st.done_merge;
  out->merges = st.merges;
  out->rounds = st.rounds;
  uint64_t a = 0;
  for (uint64_t v : att) a += v;
  out->attempts = a;
  for (int w = 0; w < I.h; ++w) {
    if (stage) stage[w] = ws[w].stage;
    if (frozen) frozen[w] = ws[w].frozen;
    if (lnf) lnf[w] = ws[w].lnf;
  }
  return REWL_OK;
}

int rewl_running(rewl_ctx* c, int32_t* n_running) {
  if (!c || !n_running) return REWL_E_INVAL;
  std::vector<InstState> st(c->lo.inst.size());
  int rc = d2h(c, st.data(), c->P.ist, st.size());
  if (rc) return rc;
  int32_t r = 0;
  for (const InstState& s : st) r += (s.done || s.error) ? 0 : 1;
  *n_running = r;
  return REWL_OK;
}

int rewl_get_geometry(rewl_ctx* c, int32_t instance, int32_t* N, int32_t* nbins, int32_t* binw,
                      int32_t* emin, int32_t* h, int32_t* m, int32_t* first_slot, int32_t* win_lo,
                      int32_t* win_hi) {
  if (!c || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  const InstDesc& I = c->lo.inst[instance];
  if (N) *N = I.N;
  if (nbins) *nbins = I.nbins;
  if (binw) *binw = I.binw;
  if (emin) *emin = I.emin;
  if (h) *h = I.h;
  if (m) *m = I.m;
  if (first_slot) *first_slot = I.slot_base;
  for (int w = 0; w < I.h; ++w) {
    if (win_lo) win_lo[w] = c->lo.win[I.win_base + w].lo;
    if (win_hi) win_hi[w] = c->lo.win[I.win_base + w].hi;
  }
  return REWL_OK;
}

int rewl_get_walker(rewl_ctx* c, int32_t instance, int32_t slot, int8_t* spins, int32_t* energy,
                    uint32_t* H, double* lng, uint64_t* attempts, int32_t* config_id) {
  if (!c || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  const InstDesc& I = c->lo.inst[instance];
  if (slot < 0 || slot >= I.W) return REWL_E_INVAL;
  const int g = I.slot_base + slot;
  const WinDesc& W = c->lo.win[I.win_base + slot / I.m];
  const int64_t base = W.lng_base + (int64_t)(slot % I.m) * W.nb;
  int32_t cfg = 0;
  int rc = d2h(c, &cfg, c->P.cfg + g, 1);
  if (rc) return rc;
  if (config_id) *config_id = cfg - I.slot_base;
  if (spins) rc = d2h(c, spins, c->P.spins + I.spin_base + (int64_t)(cfg - I.slot_base) * I.npad, (size_t)I.N);
  if (!rc && energy) rc = d2h(c, energy, c->P.E + g, 1);
  if (!rc && attempts) rc = d2h(c, attempts, c->P.att + g, 1);
  if (!rc && H) rc = d2h(c, H, c->P.H + base, (size_t)W.nb);
  if (!rc && lng) {
    if (c->lo.prec == REWL_FP64) {
      rc = d2h(c, lng, c->P.lng + base, (size_t)W.nb);
    } else {
      std::vector<float> hi(W.nb), lo(W.nb);
      rc = d2h(c, hi.data(), c->P.lhi + base, (size_t)W.nb);
      if (!rc) rc = d2h(c, lo.data(), c->P.llo + base, (size_t)W.nb);
      for (int j = 0; j < W.nb && !rc; ++j) lng[j] = (double)hi[j] + (double)lo[j];
    }
  }
  return rc;
}

int rewl_locate_walker(rewl_ctx* c, int32_t instance, int32_t slot, size_t* energy_off,
                       size_t* H_off, size_t* lng_off, int32_t* n_bins) {
  if (!c || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  const InstDesc& I = c->lo.inst[instance];
  if (slot < 0 || slot >= I.W) return REWL_E_INVAL;
  const Layout& L = c->lo;
  const WinDesc& W = L.win[I.win_base + slot / I.m];
  const size_t row = (size_t)(W.lng_base + (int64_t)(slot % I.m) * W.nb);
  if (energy_off) *energy_off = L.o_E + sizeof(int32_t) * (size_t)(I.slot_base + slot);
  if (H_off) *H_off = L.o_H + sizeof(uint32_t) * row;
  if (lng_off) *lng_off = L.prec == REWL_FP64 ? L.o_lng + sizeof(double) * row : L.o_lhi + sizeof(float) * row;
  if (n_bins) *n_bins = W.nb;
  return REWL_OK;
}

int rewl_get_walker_f32(rewl_ctx* c, int32_t instance, int32_t slot, float* hi, float* lo) {
  if (!c || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  if (c->lo.prec != REWL_FP32C) return REWL_E_STATE;
  const InstDesc& I = c->lo.inst[instance];
  if (slot < 0 || slot >= I.W) return REWL_E_INVAL;
  const WinDesc& W = c->lo.win[I.win_base + slot / I.m];
  const int64_t base = W.lng_base + (int64_t)(slot % I.m) * W.nb;
  int rc = d2h(c, hi, c->P.lhi + base, (size_t)W.nb);
  if (!rc) rc = d2h(c, lo, c->P.llo + base, (size_t)W.nb);
  return rc;
}

int rewl_get_visited(rewl_ctx* c, int32_t instance, int32_t window, uint8_t* mask) {
  if (!c || !mask || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  const InstDesc& I = c->lo.inst[instance];
  if (window < 0 || window >= I.h) return REWL_E_INVAL;
  const WinDesc& W = c->lo.win[I.win_base + window];
  return d2h(c, mask, c->P.U + W.u_base, (size_t)W.nb);
}

int rewl_get_exchange_stats(rewl_ctx* c, int32_t instance, uint64_t* tries, uint64_t* in_range,
                            uint64_t* accepts) {
  if (!c || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  const InstDesc& I = c->lo.inst[instance];
  std::vector<uint64_t> xs(3 * (size_t)I.h);
  int rc = d2h(c, xs.data(), c->P.xstats + 3 * (size_t)I.win_base, xs.size());
  if (rc) return rc;
  for (int w = 0; w < I.h; ++w) {
    if (tries) tries[w] = xs[3 * w];
    if (in_range) in_range[w] = xs[3 * w + 1];
    if (accepts) accepts[w] = xs[3 * w + 2];
  }
  return REWL_OK;
}

int rewl_get_lng(rewl_ctx* c, int32_t instance, int32_t which, double* out, int32_t capacity,
                 int32_t* n_bins_out, int32_t* joins) {
  if (!c || !out || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  if (which != 0 && which != 1) return REWL_E_INVAL;
  const InstDesc& I = c->lo.inst[instance];
  if (n_bins_out) *n_bins_out = I.nbins;
  if (capacity < I.nbins) return REWL_E_INVAL;
  int rc = hip_rc(launch_join(c->P, instance, which == 0, c->stream));
  if (rc) return rc;
  rc = d2h(c, out, c->P.R + I.r_base, (size_t)I.nbins);
  if (!rc && joins && I.h > 1) rc = d2h(c, joins, c->P.joins + I.win_base + 1, (size_t)(I.h - 1));
  return rc;
}

int rewl_get_schedule(rewl_ctx* c, int32_t instance, int32_t* phase, int64_t* stage_merge) {
  if (!c || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  const InstDesc& I = c->lo.inst[instance];
  int rc = REWL_OK;
  if (phase) {
    std::vector<WinState> ws(I.h);
    rc = d2h(c, ws.data(), c->P.wst + I.win_base, (size_t)I.h);
    for (int w = 0; w < I.h && !rc; ++w) phase[w] = ws[w].phase;
  }
  if (!rc && stage_merge)
    rc = d2h(c, stage_merge, c->P.stage_merge + (int64_t)I.win_base * kMaxStages,
             (size_t)I.h * kMaxStages);
  return rc;
}

int rewl_get_piece(rewl_ctx* c, int32_t instance, int32_t slot, double* lng) {
  if (!c || !lng || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  const InstDesc& I = c->lo.inst[instance];
  if (slot < 0 || slot >= I.W) return REWL_E_INVAL;
  const WinDesc& W = c->lo.win[I.win_base + slot / I.m];
  return d2h(c, lng, c->P.pieces + W.lng_base + (int64_t)(slot % I.m) * W.nb, (size_t)W.nb);
}

int rewl_jackknife(rewl_ctx* c, int32_t instance, double* mean, double* err, int32_t capacity,
                   int32_t* n_bins_out) {
  if (!c || !mean || !err || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  const InstDesc& I = c->lo.inst[instance];
  if (n_bins_out) *n_bins_out = I.nbins;
  if (capacity < I.nbins) return REWL_E_INVAL;
  if (I.m < 2) return REWL_E_STATE;
  InstState st;
  int rc = d2h(c, &st, c->P.ist + instance, 1);
  if (rc) return rc;
  if (!st.done) return REWL_E_STATE;
  rc = hip_rc(launch_jackknife(c->P, instance, c->P.rep + I.rep_base, c->P.jk, c->stream));
  if (!rc) rc = d2h(c, mean, c->P.jk + (int64_t)I.m * I.nbins, (size_t)I.nbins);
  if (!rc) rc = d2h(c, err, c->P.jk + (int64_t)(I.m + 1) * I.nbins, (size_t)I.nbins);
  return rc;
}

int rewl_jackknife_noalloc(rewl_ctx* c, int32_t instance, double* mean, double* err,
                           int32_t capacity, int32_t* n_bins_out) {
  if (!c || !mean || !err || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  const InstDesc& I = c->lo.inst[instance];
  if (n_bins_out) *n_bins_out = I.nbins;
  if (capacity < I.nbins) return REWL_E_INVAL;
  if (I.m < 2) return REWL_E_STATE;
  // representatives first, then the (m + 2) x nbins rows
  size_t reps = 0;
  for (int w = 0; w < I.h; ++w) reps += (size_t)c->lo.win[I.win_base + w].nb;
  const size_t rows_at = (reps + 31) / 32 * 32;  // 256-byte aligned rows
  if (rows_at + (size_t)(I.m + 2) * (size_t)I.nbins > kScratchDoubles) return REWL_E_NOMEM;
  if (!c->scratch) return REWL_E_HIP;
  InstState st;
  int rc = d2h(c, &st, c->P.ist + instance, 1);
  if (rc) return rc;
  if (!st.done) return REWL_E_STATE;
  double* jk = c->scratch + rows_at;
  rc = hip_rc(launch_jackknife(c->P, instance, c->scratch, jk, c->stream));
  if (!rc) rc = d2h(c, mean, jk + (int64_t)I.m * I.nbins, (size_t)I.nbins);
  if (!rc) rc = d2h(c, err, jk + (int64_t)(I.m + 1) * I.nbins, (size_t)I.nbins);
  return rc;
}

int rewl_thermo(rewl_ctx* c, int32_t instance, const double* T, int32_t nT, double* E_mean,
                double* C_v) {
  if (!c || !T || instance < 0 || instance >= (int32_t)c->lo.inst.size()) return REWL_E_INVAL;
  if (nT < 1 || nT > kMaxTemps) return REWL_E_INVAL;
  for (int i = 0; i < nT; ++i)
    if (!(T[i] > 0.0)) return REWL_E_INVAL;
  int rc = hip_rc(launch_join(c->P, instance, 1, c->stream));
  if (rc) return rc;
  rc = hip_rc(hipMemcpyAsync(c->P.thermo, T, sizeof(double) * nT, hipMemcpyHostToDevice, c->stream));
  if (rc) return rc;
  rc = hip_rc(launch_thermo(c->P, instance, nT, c->stream));
  if (rc) return rc;
  rc = d2h(c, E_mean, c->P.thermo + kMaxTemps, (size_t)nT);
  if (!rc) rc = d2h(c, C_v, c->P.thermo + 2 * kMaxTemps, (size_t)nT);
  return rc;
}

int rewl_checkpoint(rewl_ctx* c, void* buf, size_t cap, size_t* used) {
  if (!c) return REWL_E_INVAL;
  const size_t need = 2 * sizeof(uint64_t) + c->lo.total;
  if (used) *used = need;
  if (!buf) return REWL_OK;
  if (cap < need) return REWL_E_NOMEM;
  uint64_t hdr[2] = {kCkptMagic, (uint64_t)c->lo.total};
  memcpy(buf, hdr, sizeof(hdr));
  return d2h(c, static_cast<unsigned char*>(buf) + sizeof(hdr), c->ws, c->lo.total);
}

int rewl_restore(rewl_ctx* c, const void* buf, size_t n) {
  if (!c || !buf) return REWL_E_INVAL;
  uint64_t hdr[2];
  if (n < sizeof(hdr)) return REWL_E_FORMAT;
  memcpy(hdr, buf, sizeof(hdr));
  if (hdr[0] != kCkptMagic || hdr[1] != (uint64_t)c->lo.total || n != sizeof(hdr) + c->lo.total)
    return REWL_E_FORMAT;
  // The descriptors in the blob must describe this context's layout.
  const unsigned char* p = static_cast<const unsigned char*>(buf) + sizeof(hdr);
  const Layout& L = c->lo;
  if (memcmp(p + L.o_inst, L.inst.data(), sizeof(InstDesc) * L.inst.size()) != 0 ||
      memcmp(p + L.o_win, L.win.data(), sizeof(WinDesc) * L.win.size()) != 0)
    return REWL_E_FORMAT;
  int rc = hip_rc(hipMemcpyAsync(c->ws, p, L.total, hipMemcpyHostToDevice, c->stream));
  // the launch plan belongs to this context, not to the blob
  if (!rc)
    rc = hip_rc(hipMemcpyAsync(c->ws + L.o_wg, c->plan.wg.data(), sizeof(WgDesc) * c->plan.wg.size(),
                               hipMemcpyHostToDevice, c->stream));
  if (!rc) rc = sync(c);
  return rc;
}

int rewl_destroy(rewl_ctx* c) {
  if (!c) return REWL_E_INVAL;
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  destroy_side_streams(c);
  delete c;
  return REWL_OK;
}

const char* rewl_strerror(int code) {
  switch (code) {
    case REWL_OK: return "ok";
    case REWL_E_INVAL: return "invalid argument";
    case REWL_E_NOMEM: return "workspace or buffer too small";
    case REWL_E_HIP: return "HIP runtime error";
    case REWL_E_NONFINITE: return "non-finite ln g";
    case REWL_E_OVERFLOW: return "histogram overflow";
    case REWL_E_STATE: return "call not valid in this state";
    case REWL_E_WARMUP: return "walker could not reach its window";
    case REWL_E_FORMAT: return "checkpoint does not match this context";
    default: return "unknown error";
  }
}

}  // extern "C"
