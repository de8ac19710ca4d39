// Internal layout shared by the REWL kernels and the host-side C-ABI.
//
// All simulation state lives in one caller-provided device workspace.  The
// host computes the layout once (rewl_init) and passes device pointers to the
// kernels in a DevPtrs block.  Walker slots, windows and configurations are
// numbered globally over the batch of instances; instance i owns slots
// [slot_base, slot_base + h*m) and windows [win_base, win_base + h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rewl {

constexpr int kMaxStages = 64;    // stage bookkeeping per window
constexpr int kMaxWalkersPerWindow = 64;
constexpr int kMaxL = 64;
constexpr int kSweepWave = 64;    // walkers' wavefront of a sweep workgroup
constexpr int kRngChunk = 16;     // attempts per hand-over of the RNG producer
constexpr int kMaxTemps = 16384;  // rewl_thermo temperatures per call
// Allocation-free jackknife: doubles of the per-GPU device array that holds
// one instance's window representatives and (m + 2) x nbins leave-one-out
// rows (4 MiB), and the device ordinals it serves.
constexpr size_t kScratchDoubles = (size_t)1 << 19;
constexpr int kMaxDevices = 64;

enum Model : int32_t { kIsing = 0, kPotts = 1 };
enum Prec : int32_t { kFP64 = 0, kFP32C = 1 };
enum Schedule : int32_t { kHalving = 0, kOneOverT = 1 };
enum Tag : uint32_t { kTagMC = 0, kTagPerm = 1, kTagAcc = 2, kTagWarm = 3, kTagInit = 4 };

struct InstDesc {
  int32_t model, L, N, q;
  int32_t binw, binw_shift, emin, nbins;
  int32_t h, m, W, inst;
  int32_t slot_base, win_base, flat_num, flat_den;
  int32_t npad;          // bytes per stored configuration (multiple of 16)
  int32_t nbmax;         // largest window of this instance, bins
  int32_t r_base;        // offset of this instance's joined ln g in the R / out arrays
  int32_t rep_base;      // offset of its window representatives in rep[]
  int64_t spin_base;     // byte offset of configuration 0 of this instance
  double lnf_final;
  uint32_t key0, key1;
  int32_t schedule;      // kHalving or kOneOverT
};

struct WinDesc {
  int32_t lo, hi, nb, inst;
  int64_t lng_base;      // element offset of walker k = 0, bin lo of this window
  int32_t u_base;        // offset of the visited mask
  int32_t rep_off;       // offset of the representative within rep[]
};

struct WinState {
  double lnf;
  int32_t stage, frozen;
  int32_t phase;         // 1/t schedule: 0 = halving phase, 1 = ln f = 1/t
  int32_t pad;
};

struct InstState {
  int32_t done, error;
  int64_t done_merge;
  int64_t merges;
  uint64_t rounds;
};

// A sweep workgroup: up to 64 consecutive walker slots of one instance, and
// the kernel class of that instance (0 Ising L <= 32, 1 Ising L <= 64, 2 Potts).
struct WgDesc {
  int32_t inst, slot_first, count, cls;
};

struct DevPtrs {
  const InstDesc* inst;
  const WinDesc* win;
  const WgDesc* wg;
  InstState* ist;
  WinState* wst;
  int64_t* stage_merge;      // [windows][kMaxStages]
  uint64_t* xstats;          // [windows][3]: tries, in-range, accepts
  int32_t* cfg;              // [slots] configuration carried by each slot
  int32_t* E;                // [slots] energy of that configuration
  uint64_t* att;             // [slots] MC attempt counter
  uint64_t* watt;            // [slots] warm-up attempt counter
  int8_t* spins;             // configurations, npad bytes each
  double* lng;               // FP64 ln g, [sum over windows of m*nb]
  float* lhi;                // FP32C two-float ln g
  float* llo;
  uint32_t* H;               // histograms, same indexing as ln g
  double* pieces;            // ln g of every walker just before its window froze
  uint8_t* U;                // visited-union masks per window
  double* rep;               // window representatives for joining
  double* R;                 // joined ln g per instance
  double* thermo;            // [3][kMaxTemps]: T, <E>, C_V
  int32_t* joins;            // [windows] join bin of (w-1, w)
  double* jk;                // jackknife scratch: (m + 2) x nbins of one instance
  int32_t n_inst, n_win, n_slots, n_wg;
  int32_t prec;
  int32_t pad;
};

// Launch shape of one sweep kernel class (Ising L <= 32, Ising L <= 64,
// Potts): lanes per LDS row (walkers per workgroup), 32-bit lattice words
// per lane, ln g / H page rows per lane, first workgroup in the table, for
// Potts whether spins are kept as 4-bit nibbles (else bytes), and whether
// the workgroup keeps a table of every site's neighbours in LDS (8 bytes
// per site after the page; nibble lattices).
struct SweepShape {
  int32_t stride, nw, page, wg_offset, nib, tab;
};

// Launchers (kernels TU).  All enqueue on `s` and return the launch status.
hipError_t launch_init(const DevPtrs& P, hipStream_t s);
// One sweep kernel class: 0 = Ising L <= 32, 1 = Ising 32 < L <= 64,
// 2 = Potts; n_wg workgroups starting at sh.wg_offset of the table;
// producer: a second wavefront per workgroup computes the random numbers.
hipError_t launch_sweep_class(const DevPtrs& P, int cls, SweepShape sh, int32_t n_wg, int64_t flips,
                              size_t lds_bytes, bool producer, hipStream_t s);
// Every class in one launch (k_sweep_fused): n_wg entries of the table from
// 0, class shapes sh[0..2], lds_bytes of the largest class.
hipError_t launch_sweep_fused(const DevPtrs& P, const SweepShape sh[3], int32_t n_wg, int64_t flips,
                              size_t lds_bytes, bool producer, hipStream_t s);
hipError_t launch_merge(const DevPtrs& P, hipStream_t s);
hipError_t launch_exchange(const DevPtrs& P, hipStream_t s);
hipError_t launch_join(const DevPtrs& P, int32_t instance, int32_t normalise, hipStream_t s);
// Leave-one-out joins of an instance's frozen pieces, with the instance's
// window representatives in rep (sum of its window sizes) and the rows in jk
// ((m + 2) x nbins); mean and error land in rows m and m + 1.
hipError_t launch_jackknife(const DevPtrs& P, int32_t instance, double* rep, double* jk,
                            hipStream_t s);
// Device address, on the current GPU, of the allocation-free jackknife's
// kScratchDoubles-double array (looked up once per device).
hipError_t scratch_address(double** out);
hipError_t launch_thermo(const DevPtrs& P, int32_t instance, int32_t nT, hipStream_t s);
hipError_t prepare_sweep_lds(size_t lds_bytes);

}  // namespace rewl
