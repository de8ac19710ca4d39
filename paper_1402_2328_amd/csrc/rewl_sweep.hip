// The REWL hot path on gfx950: Wang-Landau sweeps, one walker per lane.
//
// Each workgroup is one 64-lane wavefront holding up to 64 walkers of one
// instance.  For the duration of a launch every walker keeps in LDS
//   * its lattice: Ising spins as bit rows (one 32-bit word per row for
//     L <= 32, two for L <= 64), Potts spins as 4-bit nibbles (q <= 16) or
//     bytes;
//   * a page of PG = 2^k bins of its ln g window, direct-mapped (bin b lives
//     in slot b mod PG), with the histogram increments H gathered since the
//     launch began.  Walkers move at most D bins per attempt (D = 2 for
//     Ising and q = 2 Potts, 4 for q >= 3 Potts); the page always covers
//     [bin - 2D, bin + 2D] inside the window and follows the walker by at
//     most D bins per move: the bin that leaves is written back (ln g
//     stored, its H increments added to the histogram in device memory) and
//     the bin that enters shares its slot; the entering ln g is loaded into
//     registers and committed one attempt later, since it cannot be reached
//     before then, so the load has a whole attempt to arrive (the leaving
//     bin is read out of LDS at the shift and written back one attempt
//     later as well).  Windows of at most PG bins live in LDS entirely.
// With nibble Potts lattices the workgroup also keeps, once for all its
// walkers, a table of every site's four neighbours (lattice word and nibble
// offset of each).
// Four compile-time copies of the attempt loop serve any L, L a power of
// two, Ising L = 32 (one word per row, neighbours by word rotation) and
// nibble Potts lattices with the neighbour table.
// LDS is interleaved by lane: element e of lane l sits at e * S + l (S =
// lanes per workgroup), so the 32-bit words that one instruction touches
// across the wavefront fall into consecutive banks.  Random numbers come
// from Philox4x32-10 keyed by (walker slot, attempt), so results do not
// depend on the walker-to-lane mapping, page size or launch shape.
#include <math.h>

#include <type_traits>

#include "rewl_device.h"
#include "rewl_internal.h"

namespace rewl {

// Pins a Philox block in registers at this point of the program: an empty
// asm statement (no instruction) that takes the four words as in/out
// operands, so the compiler can neither sink the rounds that produce them
// below it nor merge slices across it.
#define REWL_PIN4(v) asm volatile("" : "+v"((v).x), "+v"((v).y), "+v"((v).z), "+v"((v).w))

// Element at a 32-bit byte offset from a wave-uniform base pointer (the
// scalar-base addressing mode of global memory instructions).
template <typename T>
__device__ __forceinline__ T* at_off(T* base, uint32_t byte_off) {
  return reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(base) + byte_off);
}

// Potts proposal s0 -> v: the new value s0 + 1 + u (u < q - 1) taken
// modulo q by one unsigned minimum (v - q wraps round when v < q).
__device__ __forceinline__ int potts_wrap(int v, int q) {
  return (int)min((uint32_t)v, (uint32_t)(v - q));
}

// Energy change / J of a Potts move s0 -> v with neighbours a, b, c, d:
// (neighbours equal to s0) - (neighbours equal to v).  The four values are
// packed one per BITS-bit field (BITS = 4 for q <= 16, else 8); XOR with s
// copied into every field leaves a field zero exactly where the neighbour
// equals s, and OR-folding each field into its top bit (shift-or by
// BITS/2, .., 1 within the field) marks the fields that are not zero.  So
// the change is (nonzero fields for v) - (nonzero fields for s0), without
// compares.
template <int BITS>
__device__ __forceinline__ int potts_de(int a, int b, int c, int d, int s0, int v) {
  constexpr uint32_t rep = BITS == 4 ? 0x1111u : 0x01010101u;
  constexpr uint32_t top = BITS == 4 ? 0x8888u : 0x80808080u;
  const uint32_t n = (uint32_t)a | ((uint32_t)b << BITS) | ((uint32_t)c << (2 * BITS)) |
                     ((uint32_t)d << (3 * BITS));
  auto nonzero_fields = [&](uint32_t x) {
    if constexpr (BITS == 8) x |= x << 4;
    x |= x << 2;
    x |= x << 1;
    return __builtin_popcount(x & top);
  };
  // rep has 25 bits for BITS = 8, beyond a 24-bit multiply
  auto spread = [&](int x) { return BITS == 4 ? __mul24((uint32_t)x, rep) : (uint32_t)x * rep; };
  return nonzero_fields(n ^ spread(v)) - nonzero_fields(n ^ spread(s0));
}

// PROD: the workgroup has a second wavefront that computes the Philox
// blocks of the walkers' coming attempts, kRngChunk at a time, into a
// double buffer in LDS (chunk c in half c mod 2) while the walker wavefront
// consumes the previous chunk; one workgroup barrier per chunk hands over.
// This takes the RNG off the walkers' serial chain when few walkers share
// the chip; the blocks are the ones the walkers would compute themselves.
// The sweep of workgroup-table entry wgi, with the launch's dynamic LDS.
template <int MODEL, int PREC, int ROWW, bool PROD>
__device__ __forceinline__ void sweep_body(const DevPtrs& P, const SweepShape& sh, int64_t flips, int wgi,
                                           unsigned char* lds) {
  const WgDesc wg = P.wg[wgi];
  const InstDesc& Ig = P.inst[wg.inst];
  const int S = sh.stride;
  const int NWL = sh.nw;   // lattice words per lane
  const int PG = sh.page;  // page slots per lane, a power of two
  const int PM = PG - 1;
  const int tid = threadIdx.x;
  const int lane = tid & (kSweepWave - 1);
  // Potts nibble lattices: a table of every site's four neighbours, shared
  // by the workgroup, 8 bytes per site after the page; then the RNG double
  // buffer [2][kRngChunk][S] at the next 16-byte boundary (its reads are 16
  // bytes wide), then a flag word
  const bool use_tab = MODEL == kPotts && sh.tab != 0;
  const size_t tab_off = ((size_t)4 * NWL * S + (size_t)12 * PG * S + 7) & ~(size_t)7;
  uint2* tab = reinterpret_cast<uint2*>(lds + tab_off);
  const size_t tab_end = tab_off + (use_tab ? (size_t)8 * Ig.N : 0);
  uint4* rbuf = reinterpret_cast<uint4*>(lds + ((tab_end + 15) & ~(size_t)15));
  bool skip = P.ist[wg.inst].done || P.ist[wg.inst].error;
  if (PROD) {
    // one decision for both wavefronts: both must reach every barrier
    int* flag = reinterpret_cast<int*>(rbuf + (size_t)2 * kRngChunk * S);
    if (tid == 0) *flag = skip ? 1 : 0;
    __syncthreads();
    skip = *flag != 0;
  }
  if (skip) return;
  if (use_tab) {
    // entry of site s = y L + x: for its right, left, lower and upper
    // neighbours the lattice word (9 bits, n >> 3) and the bit offset of
    // the nibble (5 bits, 4 (n & 7)), 14 bits each, two per 32-bit word
    const int Lt = Ig.L;
    for (int s = tid; s < Ig.N; s += (int)blockDim.x) {
      const int y = s / Lt, x = s - y * Lt;
      const int nr = y * Lt + (x + 1 == Lt ? 0 : x + 1), nl = y * Lt + (x == 0 ? Lt - 1 : x - 1);
      const int nd = (y + 1 == Lt ? 0 : y + 1) * Lt + x, nu = (y == 0 ? Lt - 1 : y - 1) * Lt + x;
      auto code = [](int n) { return (uint32_t)(n >> 3) | ((uint32_t)(n & 7) << 11); };
      tab[s] = make_uint2(code(nr) | code(nl) << 14, code(nd) | code(nu) << 14);
    }
    __syncthreads();
  }
  const bool active = lane < wg.count;
  const int64_t nchunks = (flips + kRngChunk - 1) / kRngChunk;
  uint32_t* lat = reinterpret_cast<uint32_t*>(lds);                           // [NWL][S]
  unsigned char* latb = lds;                                                   // byte view (Potts)
  // Potts spins: 4-bit nibbles (8 per word; every q <= 16) or bytes
  unsigned char* pg = lds + (size_t)4 * NWL * S;
  double* plg = reinterpret_cast<double*>(pg);                                 // [PG][S] FP64
  float* plh = reinterpret_cast<float*>(pg);                                   // [PG][S] FP32C hi
  float* pll = plh + (size_t)PG * S;                                           // [PG][S] FP32C lo
  uint32_t* pH = reinterpret_cast<uint32_t*>(pg + (size_t)8 * PG * S);         // [PG][S]

  const int L = Ig.L, N = Ig.N, q = Ig.q, bshift = Ig.binw_shift;
  const bool nib = MODEL == kPotts && sh.nib != 0;
  const uint32_t k0 = Ig.key0, k1 = Ig.key1;
  const uint32_t tagw = kTagMC | ((uint32_t)Ig.inst << 8);
  const int D = (MODEL == kPotts && bshift == 0) ? 4 : 2;  // largest bin step of one move
  const int M = 2 * D;
  // row and column of a site: shifts and masks when L is a power of two
  const bool pow2 = (L & (L - 1)) == 0;
  const int Lm = L - 1;
  const int lgL = 31 - __builtin_clz((unsigned)L);

  if (PROD && tid >= kSweepWave) {
    // ---- RNG producer ----
    const int gp = wg.slot_first + lane;
    const int locp = gp - Ig.slot_base;
    const uint64_t att0 = active ? P.att[gp] : 0;
    auto fill = [&](int64_t c) {
      uint4* dst = rbuf + (size_t)(c & 1) * kRngChunk * S + lane;
      const int n = (flips - c * kRngChunk) < kRngChunk ? (int)(flips - c * kRngChunk) : kRngChunk;
      for (int i = 0; i < n; ++i) {
        const uint64_t a = att0 + (uint64_t)(c * kRngChunk + i);
        dst[(size_t)i * S] = philox10(make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)locp, tagw), k0, k1);
      }
    };
    if (active && nchunks > 0) fill(0);
    __syncthreads();
    for (int64_t c = 0; c < nchunks; ++c) {
      if (active && c + 1 < nchunks) fill(c + 1);
      __syncthreads();
    }
    return;
  }
  if (!active) return;
  const int g = wg.slot_first + lane;
  const int loc = g - Ig.slot_base;
  const int w = loc / Ig.m;
  const int k = loc - w * Ig.m;
  const WinDesc W = P.win[Ig.win_base + w];
  const WinState WS = P.wst[Ig.win_base + w];
  const int lo = W.lo, hi = W.hi, nb = W.nb;
  const bool frozen = WS.frozen != 0;
  const double lnf = WS.lnf;
  const float lnf32 = (float)WS.lnf;
  const double lnf_eff = frozen ? 0.0 : lnf;
  const uint32_t h_inc = frozen ? 0u : 1u;

  // The walkers of a workgroup are consecutive slots of one instance, so
  // their ln g / H rows form one span that starts at the row of the first
  // walker; bins are addressed by 32-bit offsets from that base.
  const int loc0 = wg.slot_first - Ig.slot_base;
  const int w0 = loc0 / Ig.m;
  const WinDesc W0 = P.win[Ig.win_base + w0];
  const int64_t gb0 = W0.lng_base + (int64_t)(loc0 - w0 * Ig.m) * W0.nb;
  const uint32_t eoff = (uint32_t)(W.lng_base + (int64_t)k * nb - gb0) - (uint32_t)lo;  // + bin
  double* const lngw = PREC == kFP64 ? P.lng + gb0 : nullptr;
  float* const lhw = PREC == kFP64 ? nullptr : P.lhi + gb0;
  float* const llw = PREC == kFP64 ? nullptr : P.llo + gb0;
  uint32_t* const Hw = P.H + gb0;

  // the energy is tracked as its bin: E = emin + bin * binw
  uint64_t att = P.att[g];
  int bin = (P.E[g] - Ig.emin) >> bshift;
  if (bin < lo || bin > hi) {
    // only reachable through corrupted state: flag the instance and keep
    // every access inside the window (the instance's results are void)
    atomicMin(&P.ist[wg.inst].error, -6);
    bin = bin < lo ? lo : hi;
  }

  // ---- stage in the lattice ----
  const int cfg = P.cfg[g];
  int8_t* gsp = P.spins + Ig.spin_base + (int64_t)(cfg - Ig.slot_base) * Ig.npad;
  if (MODEL == kIsing) {
    for (int y = 0; y < L; ++y) {
      for (int part = 0; part < ROWW; ++part) {
        uint32_t word = 0;
        const int x0 = part * 32;
        const int xe = (L - x0) < 32 ? (L - x0) : 32;
        for (int b = 0; b < xe; ++b) word |= (uint32_t)(gsp[y * L + x0 + b] > 0) << b;
        lat[(y * ROWW + part) * S + lane] = word;
      }
    }
  } else if (nib) {
    for (int i = 0; i < ((N + 7) >> 3); ++i) {
      uint32_t word = 0;
      for (int b = 0; b < 8 && 8 * i + b < N; ++b) word |= (uint32_t)(uint8_t)gsp[8 * i + b] << (4 * b);
      lat[i * S + lane] = word;
    }
  } else {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(gsp);
    const int nwi = (N + 3) >> 2;
    for (int i = 0; i < nwi; ++i) lat[i * S + lane] = src[i];
  }

  // ---- page: bins [base, base + cnt) of the window, slot of bin b = b & PM
  const bool paged = nb > PG;
  int base = lo;
  if (paged) {
    base = bin - (PG >> 1);
    base = base < lo ? lo : base;
    base = base > hi - PM ? hi - PM : base;
  }
  const int cnt = paged ? PG : nb;
  const int hi_pm = hi - PM;  // highest page start
  const int m_pm = M - PM;
  for (int i = 0; i < cnt; ++i) {
    const int b = base + i;
    const int j = __mul24(b & PM, S) + lane;
    const uint32_t e = eoff + (uint32_t)b;
    if (PREC == kFP64) {
      plg[j] = *at_off(lngw, e << 3);
    } else {
      plh[j] = *at_off(lhw, e << 2);
      pll[j] = *at_off(llw, e << 2);
    }
    pH[j] = 0;
  }
  constexpr int DMAX = (MODEL == kPotts) ? 4 : 2;
  // Bins in flight after a page shift: for slot pend_row[i], the entering
  // bin's ln g (loaded from device memory) and the leaving bin pend_e[i]
  // with its ln g and H increments (read from LDS); both are settled one
  // attempt later, which keeps the LDS read's latency out of the shift.
  int pend_n = 0;
  int pend_row[DMAX];
  uint32_t pend_e[DMAX], ev_h[DMAX];
  double pend_l[DMAX], ev_l[DMAX];
  float pend_hi[DMAX], pend_lo[DMAX], ev_hi[DMAX], ev_lo[DMAX];
#pragma unroll
  for (int i = 0; i < DMAX; ++i) {
    pend_row[i] = 0;
    pend_e[i] = ev_h[i] = 0u;
    pend_l[i] = ev_l[i] = 0.0;
    pend_hi[i] = pend_lo[i] = ev_hi[i] = ev_lo[i] = 0.0f;
  }
  // Settles the bins in flight: the leaving bins are written back (ln g
  // stored, H increments added to the histogram in device memory) and the
  // entering bins take their slots.
  auto settle = [&]() {
#pragma unroll
    for (int i = 0; i < DMAX; ++i) {
      if (i < pend_n) {
        const int j = pend_row[i];
        if (PREC == kFP64) {
          plg[j] = pend_l[i];
        } else {
          plh[j] = pend_hi[i];
          pll[j] = pend_lo[i];
        }
        pH[j] = 0;
        const uint32_t e = pend_e[i];
        if (PREC == kFP64) {
          *at_off(lngw, e << 3) = ev_l[i];
        } else {
          *at_off(lhw, e << 2) = ev_hi[i];
          *at_off(llw, e << 2) = ev_lo[i];
        }
        atomicAdd(at_off(Hw, e << 2), ev_h[i]);
      }
    }
    pend_n = 0;
  };

  int jcur = __mul24(bin & PM, S) + lane;  // LDS row index of the current bin
  double lcur = 0.0;
  float hcur = 0.0f, lcur_lo = 0.0f;
  if (PREC == kFP64) lcur = plg[jcur];
  else {
    hcur = plh[jcur];
    lcur_lo = pll[jcur];
  }

  const int lane4 = lane * 4;
  const int S4 = S * 4;
  // addresses stay below 2^24, so 24-bit multiplies (full rate) suffice
  auto pbyte = [&](int site) { return __mul24(site >> 2, S4) + lane4 + (site & 3); };

  auto prow = [&](int row) { return __mul24(row, S) + lane; };
  auto pnib = [&](int site) { return prow(site >> 3); };  // word holding a nibble

  // Rest of an attempt once the proposal is known: ln g at the proposed
  // bin, acceptance, lattice and ln g / H update, page follow.  Without a
  // producer, the last two Philox slices of the block in flight (rn) are
  // placed beside the ln g read and the exponential.
  // bn is the proposed bin.  bn & PM always names a slot of the page, so the
  // ln g read stays in bounds when bn lies outside the window; its value is
  // then not used.
  uint2 tab_e = make_uint2(0u, 0u), tab_en = make_uint2(0u, 0u);  // neighbour table entries
  auto complete = [&](const uint4 r, uint4& rn, int bn, int nv, uint32_t wofs, uint32_t wrow,
                      uint32_t fm, int site, auto lkt, auto nbt) -> bool {
    constexpr bool NB = decltype(nbt)::value;
    constexpr bool TAB = decltype(lkt)::value == 3;
    const bool inwin = (bn >= lo) && (bn <= hi);
    const int jn = prow(bn & PM);
    bool acc;
    if (PREC == kFP64) {
      const double ln = plg[jn];
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (!PROD) {
        rn = philox_rounds<4, 7>(rn, k0, k1);
        REWL_PIN4(rn);
      }
      __builtin_amdgcn_sched_barrier(0);
      const bool a = accept64_fast(r.z, r.w, lcur - ln);
      if constexpr (!PROD) {
        rn = philox_rounds<7, 10>(rn, k0, k1);
        REWL_PIN4(rn);
        // the next attempt's neighbour table entry, read while this
        // attempt finishes
        if constexpr (TAB) tab_en = tab[__umulhi(rn.x, (uint32_t)N)];
      }
      acc = inwin && a;
      lcur = acc ? ln : lcur;
    } else {
      const float nh = plh[jn];
      const float nl = pll[jn];
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (!PROD) {
        rn = philox_rounds<4, 7>(rn, k0, k1);
        REWL_PIN4(rn);
      }
      __builtin_amdgcn_sched_barrier(0);
      const bool a = accept32_fast(r.z >> 8, (hcur - nh) + (lcur_lo - nl));
      if constexpr (!PROD) {
        rn = philox_rounds<7, 10>(rn, k0, k1);
        REWL_PIN4(rn);
        // the next attempt's neighbour table entry, read while this
        // attempt finishes
        if constexpr (TAB) tab_en = tab[__umulhi(rn.x, (uint32_t)N)];
      }
      acc = inwin && a;
      hcur = acc ? nh : hcur;
      lcur_lo = acc ? nl : lcur_lo;
    }
    if (MODEL == kIsing) {
      // the row word is written back either way (unchanged when rejected)
      *reinterpret_cast<uint32_t*>(lds + wofs) = acc ? wrow ^ fm : wrow;
    } else if (acc) {
      if constexpr (NB) {
        const int sh4 = (site & 7) * 4;
        *reinterpret_cast<uint32_t*>(lds + wofs) = (wrow & ~(15u << sh4)) | ((uint32_t)nv << sh4);
      } else {
        latb[pbyte(site)] = (unsigned char)nv;
      }
    }
    bin = acc ? bn : bin;
    jcur = acc ? jn : jcur;
    if (PREC == kFP64) {
      // frozen walkers add 0.0 and count 0: ln g >= +0 always, so x + 0.0
      // is x bit for bit, and the branch-free form needs no exec mask
      lcur = lcur + lnf_eff;
      plg[jcur] = lcur;
      atomicAdd(&pH[jcur], h_inc);
    } else if (!frozen) {
      // a two-float add of 0 could renormalise the pair, so frozen FP32C
      // walkers skip the update instead
      df_add1(hcur, lcur_lo, lnf32, hcur, lcur_lo);
      plh[jcur] = hcur;
      pll[jcur] = lcur_lo;
      atomicAdd(&pH[jcur], 1u);  // no-return LDS add: the lane owns this word
    }
    // settle the bins of the last shift, then follow the walker
    settle();
    if (paged) {
      // bin + M - PM is the lowest page start that still covers bin + M,
      // bin - M the highest that covers bin - M (PM >= 2M); the start then
      // stays inside [lo, hi - PM].  Both are integer medians.
      constexpr bool MA = MODEL == kIsing;  // Ising: 2 % faster; Potts: 1-2 % slower
      const int nbase = med3_i32<MA>(med3_i32<MA>(base, bin + m_pm, bin - M), lo, hi_pm);
      const int sft = nbase - base;  // -D..D
      const bool up = sft > 0;
      const int shn = up ? sft : -sft;
      // up: bins base, base+1, .. leave and the bins PG above them enter;
      // down: bins base+PM, base+PM-1, .. leave and the bins PG below them enter --
      // each pair shares a slot.  A frozen walker writes back its unchanged
      // ln g and no H increments.
      const int stp = up ? 1 : -1;
      const int ev0 = up ? base : base + PM;
      const int dpg = __mul24(stp, PG);
#pragma unroll
      for (int i = 0; i < DMAX; ++i) {
        if (i < shn) {
          const int ev = ev0 + i * stp;
          const uint32_t e = eoff + (uint32_t)ev;
          const uint32_t en = e + (uint32_t)dpg;
          const int j = prow(ev & PM);
          if (PREC == kFP64) {
            ev_l[i] = plg[j];
          } else {
            ev_hi[i] = plh[j];
            ev_lo[i] = pll[j];
          }
          ev_h[i] = pH[j];
          pend_e[i] = e;
          if (PREC == kFP64) {
            pend_l[i] = *at_off(lngw, en << 3);
          } else {
            pend_hi[i] = *at_off(lhw, en << 2);
            pend_lo[i] = *at_off(llw, en << 2);
          }
          pend_row[i] = j;
        }
      }
      base = nbase;
      pend_n = shn;
    }
    ++att;
    return acc;
  };

  // Software pipeline: the Philox block of attempt t+1 (it depends only on
  // the attempt counter) is computed in three slices placed in the latency
  // shadows of attempt t -- after the lattice reads are issued, after the
  // ln g read is issued, and beside the exponential.  sched_barrier keeps
  // the compiler from hoisting the slices back together.
  // One attempt with Philox block r; without a producer it also computes
  // rn, the block of the next attempt, in slices.  The lattice form LK
  // (0: any L, 1: L a power of two, 2: Ising with L = 32, one word per row,
  // 3: Potts nibbles with the neighbour table) and NB (Potts nibbles)
  // select compile-time copies of the loop, chosen
  // once per launch, so that no branch splits the attempt's scheduling
  // region.
  auto attempt = [&](const uint4 r, uint4& rn, auto lkt, auto nbt) {
    constexpr int LK = decltype(lkt)::value;
    constexpr bool P2 = LK >= 1;
    constexpr bool NB = decltype(nbt)::value;
    const uint64_t an = att + 1;
    const uint4 cn = make_uint4((uint32_t)an, (uint32_t)(an >> 32), (uint32_t)loc, tagw);
    const int site = (int)__umulhi(r.x, (uint32_t)N);
    if constexpr (LK == 2) {
      // Ising, L = 32: row y = site / 32 is one word, column x = site % 32.
      // Rotating the row right by x puts the spin at bit 0 and its right
      // neighbour at bit 1; one more rotation left puts the left neighbour
      // at bit 0 and the spin at bit 1.  Word shifts and rotations use the
      // low five bits of site, which is x.  The bin step is
      // db = (agreeing neighbours) - 2 (Delta E = 2 s sum, in bins of 4).
      const int y = site >> 5;
      const uint32_t aw = __mul24((uint32_t)y, (uint32_t)S4) + (uint32_t)lane4;
      const uint32_t ad = __mul24((uint32_t)((y + 1) & 31), (uint32_t)S4) + (uint32_t)lane4;
      const uint32_t au = __mul24((uint32_t)((y - 1) & 31), (uint32_t)S4) + (uint32_t)lane4;
      uint32_t awk = aw;
      asm volatile("" : "+v"(awk));  // keep the address for the write-back
      const uint32_t wrow = *reinterpret_cast<const uint32_t*>(lds + awk);
      const uint32_t wd = *reinterpret_cast<const uint32_t*>(lds + ad);
      const uint32_t wu = *reinterpret_cast<const uint32_t*>(lds + au);
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (!PROD) {
        rn = philox_rounds<0, 4>(cn, k0, k1);
        REWL_PIN4(rn);
      }
      __builtin_amdgcn_sched_barrier(0);
      const uint32_t fm = 1u << (site & 31);
      const uint32_t tr = __builtin_amdgcn_alignbit(wrow, wrow, (uint32_t)site);
      const uint32_t tl = __builtin_amdgcn_alignbit(tr, tr, 31u);
      const uint32_t hz = ~(tl ^ tr) & 3u;     // left and right agree with the spin
      const uint32_t vd = ~(wd ^ wrow) & fm;   // lower neighbour agrees
      const uint32_t vu = ~(wu ^ wrow) & fm;   // upper neighbour agrees
      const int bn = bin - 2 + __builtin_popcount(hz) + __builtin_popcount(vd) + __builtin_popcount(vu);
      complete(r, rn, bn, 0, awk, wrow, fm, site, lkt, nbt);
      return;
    }
    if constexpr (LK == 3) {
      // Potts nibbles with the neighbour table: the site's word and nibble
      // from the site, its neighbours' from the table entry read one
      // attempt ahead, so no row, column or wrap arithmetic
      const uint2 e = tab_e;
      // byte offset of lattice word wd of this lane: wd * 4S + 4 lane
      auto word_at = [&](uint32_t wd) {
        return *reinterpret_cast<const uint32_t*>(lds + __mul24(wd, (uint32_t)S4) + (uint32_t)lane4);
      };
      const uint32_t wofs = __mul24((uint32_t)site >> 3, (uint32_t)S4) + (uint32_t)lane4;
      const uint32_t w0 = *reinterpret_cast<const uint32_t*>(lds + wofs);
      const uint32_t w1 = word_at(__builtin_amdgcn_ubfe(e.x, 0, 9));
      const uint32_t w2 = word_at(__builtin_amdgcn_ubfe(e.x, 14, 9));
      const uint32_t w3 = word_at(__builtin_amdgcn_ubfe(e.y, 0, 9));
      const uint32_t w4 = word_at(__builtin_amdgcn_ubfe(e.y, 14, 9));
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (!PROD) {
        rn = philox_rounds<0, 4>(cn, k0, k1);
        REWL_PIN4(rn);
      }
      __builtin_amdgcn_sched_barrier(0);
      const int s0 = (int)__builtin_amdgcn_ubfe(w0, (site & 7) * 4, 4);
      const int a = (int)__builtin_amdgcn_ubfe(w1, __builtin_amdgcn_ubfe(e.x, 9, 5), 4);
      const int b = (int)__builtin_amdgcn_ubfe(w2, __builtin_amdgcn_ubfe(e.x, 23, 5), 4);
      const int c = (int)__builtin_amdgcn_ubfe(w3, __builtin_amdgcn_ubfe(e.y, 9, 5), 4);
      const int d = (int)__builtin_amdgcn_ubfe(w4, __builtin_amdgcn_ubfe(e.y, 23, 5), 4);
      const int v = potts_wrap(s0 + 1 + (int)__umulhi(r.y, (uint32_t)(q - 1)), q);
      const int dE = potts_de<4>(a, b, c, d, s0, v);
      complete(r, rn, bin + (dE >> bshift), v, wofs, w0, 0u, site, lkt, nbt);
      return;
    }
    int y, x, xr, xl, yd, yu;
    if constexpr (P2) {  // shifts and masks
      y = site >> lgL;
      x = site & Lm;
      xr = (x + 1) & Lm;
      xl = (x - 1) & Lm;
      yd = (y + 1) & Lm;
      yu = (y - 1) & Lm;
    } else {
      // site = floor(r.x N / 2^32) with N = L^2, so its row
      // floor(site / L) = floor(r.x L / 2^32): one multiply, off the chain
      // of the site itself
      y = (int)__umulhi(r.x, (uint32_t)L);
      x = site - __mul24(y, L);
      xr = (x + 1 == L) ? 0 : x + 1;
      xl = (x == 0) ? L - 1 : x - 1;
      yd = (y + 1 == L) ? 0 : y + 1;
      yu = (y == 0) ? L - 1 : y - 1;
    }
    int db, nv = 0;
    int widx = 0;
    uint32_t wrow = 0, fm = 0;
    if (MODEL == kIsing) {
      // bit b of a row word: spin at x = 32 * part + b is +1
      int s0, a, b, c, d;
      if (ROWW == 1) {
        widx = prow(y);
        wrow = lat[widx];
        const uint32_t wu = lat[prow(yu)];
        const uint32_t wd = lat[prow(yd)];
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (!PROD) {
          rn = philox_rounds<0, 4>(cn, k0, k1);
          REWL_PIN4(rn);
        }
        __builtin_amdgcn_sched_barrier(0);
        s0 = (wrow >> x) & 1;
        a = (wrow >> xr) & 1;
        b = (wrow >> xl) & 1;
        c = (wd >> x) & 1;
        d = (wu >> x) & 1;
      } else {
        const int px = x >> 5;
        const uint32_t r0 = lat[prow(2 * y)];
        const uint32_t r1 = lat[prow(2 * y + 1)];
        const uint32_t wu = lat[prow(2 * yu + px)];
        const uint32_t wd = lat[prow(2 * yd + px)];
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (!PROD) {
          rn = philox_rounds<0, 4>(cn, k0, k1);
          REWL_PIN4(rn);
        }
        __builtin_amdgcn_sched_barrier(0);
        wrow = px ? r1 : r0;
        s0 = (wrow >> (x & 31)) & 1;
        a = (((xr >> 5) ? r1 : r0) >> (xr & 31)) & 1;
        b = (((xl >> 5) ? r1 : r0) >> (xl & 31)) & 1;
        c = (wd >> (x & 31)) & 1;
        d = (wu >> (x & 31)) & 1;
        widx = prow(2 * y + px);
      }
      // sigma = 2 bit - 1: dE = 2 s0 (sum of neighbours), bin step dE / 4
      db = (2 * s0 - 1) * (a + b + c + d - 2);
      fm = 1u << (x & 31);
    } else {
      const int rowy = __mul24(y, L);
      int s0, a, b, c, d;
      if constexpr (NB) {
        const int sa = rowy + xr, sb = rowy + xl, sc = __mul24(yd, L) + x, sd = __mul24(yu, L) + x;
        widx = pnib(site);
        wrow = lat[widx];
        s0 = (int)__builtin_amdgcn_ubfe(wrow, (site & 7) * 4, 4);
        a = (int)__builtin_amdgcn_ubfe(lat[pnib(sa)], (sa & 7) * 4, 4);
        b = (int)__builtin_amdgcn_ubfe(lat[pnib(sb)], (sb & 7) * 4, 4);
        c = (int)__builtin_amdgcn_ubfe(lat[pnib(sc)], (sc & 7) * 4, 4);
        d = (int)__builtin_amdgcn_ubfe(lat[pnib(sd)], (sd & 7) * 4, 4);
      } else {
        s0 = (int)latb[pbyte(site)];
        a = (int)latb[pbyte(rowy + xr)];
        b = (int)latb[pbyte(rowy + xl)];
        c = (int)latb[pbyte(__mul24(yd, L) + x)];
        d = (int)latb[pbyte(__mul24(yu, L) + x)];
      }
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (!PROD) {
        rn = philox_rounds<0, 4>(cn, k0, k1);
        REWL_PIN4(rn);
      }
      __builtin_amdgcn_sched_barrier(0);
      const int v = potts_wrap(s0 + 1 + (int)__umulhi(r.y, (uint32_t)(q - 1)), q);
      nv = v;
      db = (NB ? potts_de<4>(a, b, c, d, s0, v) : potts_de<8>(a, b, c, d, s0, v)) >> bshift;
    }
    complete(r, rn, bin + db, nv, 4u * (uint32_t)widx, wrow, fm, site, lkt, nbt);
  };


  using T = std::true_type;
  using F = std::false_type;

  auto run = [&](auto lkt, auto nbt) {
    constexpr bool TAB = decltype(lkt)::value == 3;
    if constexpr (!PROD) {
      uint4 r = philox10(make_uint4((uint32_t)att, (uint32_t)(att >> 32), (uint32_t)loc, tagw), k0, k1);
      if constexpr (TAB) tab_e = tab[__umulhi(r.x, (uint32_t)N)];
      for (int64_t t = 0; t < flips; ++t) {
        uint4 rn;
        attempt(r, rn, lkt, nbt);
        r = rn;
        if constexpr (TAB) tab_e = tab_en;
      }
    } else {
      __syncthreads();  // chunk 0 is in the buffer
      for (int64_t c = 0; c < nchunks; ++c) {
        const uint4* src = rbuf + (size_t)(c & 1) * kRngChunk * S + lane;
        const int n = (flips - c * kRngChunk) < kRngChunk ? (int)(flips - c * kRngChunk) : kRngChunk;
        uint4 r = src[0];
        if constexpr (TAB) tab_e = tab[__umulhi(r.x, (uint32_t)N)];
        for (int i = 0; i < n; ++i) {
          const uint4 rnext = src[(size_t)(i + 1 < n ? i + 1 : i) * S];
          if constexpr (TAB) tab_en = tab[__umulhi(rnext.x, (uint32_t)N)];
          uint4 unused;
          attempt(r, unused, lkt, nbt);
          r = rnext;
          if constexpr (TAB) tab_e = tab_en;
        }
        __syncthreads();  // chunk c consumed, chunk c + 1 written
      }
    }
  };
  using L0 = std::integral_constant<int, 0>;
  using L1 = std::integral_constant<int, 1>;
  using L2 = std::integral_constant<int, 2>;
  using L3 = std::integral_constant<int, 3>;
  if (MODEL == kPotts && nib && use_tab) {
    if constexpr (MODEL == kPotts) run(L3{}, T{});
  } else if (MODEL == kPotts && nib) {
    if (pow2) run(L1{}, T{});
    else run(L0{}, T{});
  } else if (MODEL == kIsing && ROWW == 1 && L == 32) {
    if constexpr (MODEL == kIsing && ROWW == 1) run(L2{}, F{});
  } else {
    if (pow2) run(L1{}, F{});
    else run(L0{}, F{});
  }

  // ---- stage out ----
  settle();
  if (!frozen) {
    for (int i = 0; i < cnt; ++i) {
      const int b = base + i;
      const int j = prow(b & PM);
      const uint32_t e = eoff + (uint32_t)b;
      if (PREC == kFP64) {
        *at_off(lngw, e << 3) = plg[j];
      } else {
        *at_off(lhw, e << 2) = plh[j];
        *at_off(llw, e << 2) = pll[j];
      }
      const uint32_t h = pH[j];
      if (h) atomicAdd(at_off(Hw, e << 2), h);
    }
  }
  if (MODEL == kIsing) {
    for (int y = 0; y < L; ++y) {
      for (int part = 0; part < ROWW; ++part) {
        const uint32_t word = lat[(y * ROWW + part) * S + lane];
        const int x0 = part * 32;
        const int xe = (L - x0) < 32 ? (L - x0) : 32;
        for (int b = 0; b < xe; ++b) gsp[y * L + x0 + b] = ((word >> b) & 1) ? 1 : -1;
      }
    }
  } else if (nib) {
    for (int i = 0; i < ((N + 7) >> 3); ++i) {
      const uint32_t word = lat[i * S + lane];
      for (int b = 0; b < 8 && 8 * i + b < N; ++b) gsp[8 * i + b] = (int8_t)((word >> (4 * b)) & 15);
    }
  } else {
    uint32_t* dst = reinterpret_cast<uint32_t*>(gsp);
    const int nwi = (N + 3) >> 2;
    for (int i = 0; i < nwi; ++i) dst[i] = lat[i * S + lane];
  }
  P.E[g] = Ig.emin + (bin << bshift);  // every energy sits on the bin grid
  P.att[g] = att;
}

// One kernel class per launch: the class's workgroups are entries
// [sh.wg_offset, sh.wg_offset + gridDim.x) of the table.
template <int MODEL, int PREC, int ROWW, bool PROD>
__global__ __launch_bounds__(PROD ? 2 * kSweepWave : kSweepWave) void k_sweep(DevPtrs P, SweepShape sh,
                                                                                int64_t flips) {
  extern __shared__ __align__(16) unsigned char lds[];
  sweep_body<MODEL, PREC, ROWW, PROD>(P, sh, flips, sh.wg_offset + (int)blockIdx.x, lds);
}

// Every kernel class of a batch in one launch: workgroup b runs table entry
// b with the loop of its class (all its lanes take the same branch), in
// the LDS size of the largest class.  The table order decides which
// workgroups the hardware dispatches first.
template <int PREC, bool PROD>
__global__ __launch_bounds__(PROD ? 2 * kSweepWave : kSweepWave) void k_sweep_fused(DevPtrs P, SweepShape s0,
                                                                                      SweepShape s1,
                                                                                      SweepShape s2,
                                                                                      int64_t flips) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int wgi = (int)blockIdx.x;
  const int cls = P.wg[wgi].cls;
  if (cls == 0) sweep_body<kIsing, PREC, 1, PROD>(P, s0, flips, wgi, lds);
  else if (cls == 1) sweep_body<kIsing, PREC, 2, PROD>(P, s1, flips, wgi, lds);
  else sweep_body<kPotts, PREC, 0, PROD>(P, s2, flips, wgi, lds);
}

hipError_t prepare_sweep_lds(size_t lds_bytes) {
  const void* fns[] = {
      (const void*)k_sweep<kIsing, kFP64, 1, false>,  (const void*)k_sweep<kIsing, kFP64, 2, false>,
      (const void*)k_sweep<kPotts, kFP64, 0, false>,  (const void*)k_sweep<kIsing, kFP32C, 1, false>,
      (const void*)k_sweep<kIsing, kFP32C, 2, false>, (const void*)k_sweep<kPotts, kFP32C, 0, false>,
      (const void*)k_sweep<kIsing, kFP64, 1, true>,   (const void*)k_sweep<kIsing, kFP64, 2, true>,
      (const void*)k_sweep<kPotts, kFP64, 0, true>,   (const void*)k_sweep<kIsing, kFP32C, 1, true>,
      (const void*)k_sweep<kIsing, kFP32C, 2, true>,  (const void*)k_sweep<kPotts, kFP32C, 0, true>,
      (const void*)k_sweep_fused<kFP64, false>,       (const void*)k_sweep_fused<kFP64, true>,
      (const void*)k_sweep_fused<kFP32C, false>,      (const void*)k_sweep_fused<kFP32C, true>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool PROD>
void launch_class(const DevPtrs& P, int cls, SweepShape sh, dim3 grid, int64_t flips, size_t lds_bytes,
                  hipStream_t s) {
  const dim3 blk(PROD ? 2 * kSweepWave : kSweepWave);
  if (P.prec == kFP64) {
    if (cls == 0) hipLaunchKernelGGL((k_sweep<kIsing, kFP64, 1, PROD>), grid, blk, lds_bytes, s, P, sh, flips);
    if (cls == 1) hipLaunchKernelGGL((k_sweep<kIsing, kFP64, 2, PROD>), grid, blk, lds_bytes, s, P, sh, flips);
    if (cls == 2) hipLaunchKernelGGL((k_sweep<kPotts, kFP64, 0, PROD>), grid, blk, lds_bytes, s, P, sh, flips);
  } else {
    if (cls == 0) hipLaunchKernelGGL((k_sweep<kIsing, kFP32C, 1, PROD>), grid, blk, lds_bytes, s, P, sh, flips);
    if (cls == 1) hipLaunchKernelGGL((k_sweep<kIsing, kFP32C, 2, PROD>), grid, blk, lds_bytes, s, P, sh, flips);
    if (cls == 2) hipLaunchKernelGGL((k_sweep<kPotts, kFP32C, 0, PROD>), grid, blk, lds_bytes, s, P, sh, flips);
  }
}

hipError_t launch_sweep_class(const DevPtrs& P, int cls, SweepShape sh, int32_t n_wg, int64_t flips,
                              size_t lds_bytes, bool producer, hipStream_t s) {
  if (n_wg <= 0) return hipSuccess;
  if (producer) launch_class<true>(P, cls, sh, dim3(n_wg), flips, lds_bytes, s);
  else launch_class<false>(P, cls, sh, dim3(n_wg), flips, lds_bytes, s);
  return hipGetLastError();
}

hipError_t launch_sweep_fused(const DevPtrs& P, const SweepShape sh[3], int32_t n_wg, int64_t flips,
                              size_t lds_bytes, bool producer, hipStream_t s) {
  if (n_wg <= 0) return hipSuccess;
  const dim3 grid(n_wg), blk(producer ? 2 * kSweepWave : kSweepWave);
  if (P.prec == kFP64) {
    if (producer) hipLaunchKernelGGL((k_sweep_fused<kFP64, true>), grid, blk, lds_bytes, s, P, sh[0], sh[1], sh[2], flips);
    else hipLaunchKernelGGL((k_sweep_fused<kFP64, false>), grid, blk, lds_bytes, s, P, sh[0], sh[1], sh[2], flips);
  } else {
    if (producer) hipLaunchKernelGGL((k_sweep_fused<kFP32C, true>), grid, blk, lds_bytes, s, P, sh[0], sh[1], sh[2], flips);
    else hipLaunchKernelGGL((k_sweep_fused<kFP32C, false>), grid, blk, lds_bytes, s, P, sh[0], sh[1], sh[2], flips);
  }
  return hipGetLastError();
}

}  // namespace rewl
