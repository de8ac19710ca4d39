// Issue cost of the vector instruction forms the sweep kernel is built
// from, and the LDS read bandwidth, measured on the current device.  The
// sweep's roofline counts its work in full-rate lane-op slots; this measures
// what one slot costs, whether the 32 x 32 -> 64 multiplies of Philox4x32
// issue at the full rate, and the LDS bytes per clock a CU delivers.
//
// Every kernel runs 8 independent dependency chains per lane (enough to
// cover the ALU latency) over a grid of 8 wavefronts per SIMD, so the time
// is the issue time.  One output word per thread keeps the chains alive.
//
// C-ABI (measurement only, not part of the REWL library):
//   int alu_rate(int32_t iters, double* out, int32_t n_out)
// out[k] = ns per wavefront step per SIMD for form k (n_out >= 5):
//   0  v_xad_u32                       (one full-rate op per step)
//   1  v_mad_u64_u32 + v_xor_b32       (a Philox multiply and one xor)
//   2  v_mul_lo_u32 + v_mul_hi_u32 + v_xor_b32
//   3  v_fma_f64
//   4  v_bitop3_b32 (three-input xor)
//   int lds_rate(int32_t iters, double* out, int32_t n_out)
// out[k] = LDS bytes read per second over the whole chip (n_out >= 3) with
// conflict-free reads of 4, 8 and 16 B per lane (the compiler pairs the
// first two into ds_read2st64_b32 / ds_read2st64_b64; the third is
// ds_read_b128), 16 wavefronts per CU, consecutive lanes on consecutive
// elements.
// Both return 0, or -1 for bad arguments, -2 for a HIP error.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kChains = 8;
constexpr int kThreads = 256;

template <int FORM>
__global__ __launch_bounds__(kThreads) void k_rate(uint32_t* out, int iters, uint32_t seed) {
  uint32_t x[kChains];
  double d[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    x[c] = seed ^ (threadIdx.x * kChains + c) ^ (blockIdx.x << 12);
    d[c] = (double)x[c] * 0x1p-32;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (FORM == 0) {
        x[c] = (x[c] ^ 0x9E3779B9u) + (uint32_t)(c + 1);
      } else if constexpr (FORM == 1) {
        const uint64_t r = (uint64_t)x[c] * 0xD2511F53u;
        x[c] = (uint32_t)(r >> 32) ^ (uint32_t)r;
      } else if constexpr (FORM == 2) {
        const uint32_t lo = x[c] * 0xD2511F53u;
        const uint32_t hi = __umulhi(x[c], 0xD2511F53u);
        x[c] = hi ^ lo;
      } else if constexpr (FORM == 3) {
        d[c] = fma(d[c], 0.999999, 1e-7);
      } else {
        x[c] = __builtin_amdgcn_bitop3_b32(x[c], 0x9E3779B9u, (uint32_t)i, 0x96);
      }
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= x[c] ^ (uint32_t)(d[c] * 0x1p20);
  out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// LDS reads of W 32-bit words per lane: every iteration reads one 16 KB half
// of a 32 KB buffer (the two halves alternate), 64 B per lane as 16 / W
// reads at immediate offsets from one address, so that address arithmetic
// is one add per iteration; three-input xors keep every word live, and a
// compiler barrier at the top of the iteration forces the reads each time.
template <int W>
__global__ __launch_bounds__(kThreads) void k_lds(uint32_t* out, int iters) {
  constexpr int kWords = 8192;  // 32 KB
  constexpr int kRow = kThreads * W * 4;  // bytes of one read across the block
  constexpr int kReads = 16 / W;
  __shared__ __align__(16) uint32_t buf[kWords];
  for (int i = threadIdx.x; i < kWords; i += kThreads) buf[i] = (uint32_t)i * 0x9E3779B9u ^ blockIdx.x;
  __syncthreads();
  const unsigned char* base = reinterpret_cast<const unsigned char*>(buf) + threadIdx.x * W * 4;
  uint32_t acc = 0;
  for (int i = 0; i < iters; ++i) {
    asm volatile("" ::: "memory");
    const unsigned char* p = base + ((i & 1) << 14);
    uint32_t w[16];
#pragma unroll
    for (int k = 0; k < kReads; ++k) {
      if constexpr (W == 1) {
        w[k] = *reinterpret_cast<const uint32_t*>(p + k * kRow);
      } else if constexpr (W == 2) {
        const uint2 v = *reinterpret_cast<const uint2*>(p + k * kRow);
        w[2 * k] = v.x;
        w[2 * k + 1] = v.y;
      } else {
        const uint4 v = *reinterpret_cast<const uint4*>(p + k * kRow);
        w[4 * k] = v.x;
        w[4 * k + 1] = v.y;
        w[4 * k + 2] = v.z;
        w[4 * k + 3] = v.w;
      }
    }
#pragma unroll
    for (int k = 0; k < 16; k += 2) acc = __builtin_amdgcn_bitop3_b32(acc, w[k], w[k + 1], 0x96);
  }
  out[blockIdx.x * kThreads + threadIdx.x] = acc;
}

}  // namespace

extern "C" int lds_rate(int32_t iters, double* out, int32_t n_out) {
  if (iters <= 0 || !out || n_out < 3) return -1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return -2;
  const int blocks = 4 * cus;  // 16 wavefronts of 64 per CU, 128 KB of LDS
  uint32_t* buf = nullptr;
  if (hipMalloc(&buf, sizeof(uint32_t) * (size_t)blocks * kThreads) != hipSuccess) return -2;
  hipEvent_t a = nullptr, b = nullptr;
  int rc = 0;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = -2;
  for (int form = 0; form < 3 && rc == 0; ++form) {
    float best = -1.0f;
    for (int rep = 0; rep < 3 && rc == 0; ++rep) {
      if (hipEventRecord(a, 0) != hipSuccess) rc = -2;
      if (form == 0) hipLaunchKernelGGL(k_lds<1>, dim3(blocks), dim3(kThreads), 0, 0, buf, iters);
      if (form == 1) hipLaunchKernelGGL(k_lds<2>, dim3(blocks), dim3(kThreads), 0, 0, buf, iters);
      if (form == 2) hipLaunchKernelGGL(k_lds<4>, dim3(blocks), dim3(kThreads), 0, 0, buf, iters);
      if (hipGetLastError() != hipSuccess || hipEventRecord(b, 0) != hipSuccess ||
          hipEventSynchronize(b) != hipSuccess)
        rc = -2;
      float ms = 0.0f;
      if (rc == 0 && hipEventElapsedTime(&ms, a, b) != hipSuccess) rc = -2;
      if (rc == 0 && rep > 0 && (best < 0.0f || ms < best)) best = ms;
    }
    const double bytes = (double)blocks * kThreads * iters * 64.0;  // 64 B per lane and iteration
    if (rc == 0) out[form] = bytes / ((double)best * 1e-3);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(buf);
  return rc;
}

extern "C" int alu_rate(int32_t iters, double* out, int32_t n_out) {
  if (iters <= 0 || !out || n_out < 5) return -1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return -2;
  const int simds = 4 * cus;
  const int blocks = 2 * simds;  // 8 wavefronts of 64 per SIMD
  uint32_t* buf = nullptr;
  if (hipMalloc(&buf, sizeof(uint32_t) * (size_t)blocks * kThreads) != hipSuccess) return -2;
  hipEvent_t a = nullptr, b = nullptr;
  int rc = 0;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) rc = -2;
  for (int form = 0; form < 5 && rc == 0; ++form) {
    float best = -1.0f;
    for (int rep = 0; rep < 3 && rc == 0; ++rep) {  // the first run warms the clocks
      if (hipEventRecord(a, 0) != hipSuccess) rc = -2;
      switch (form) {
        case 0: hipLaunchKernelGGL(k_rate<0>, dim3(blocks), dim3(kThreads), 0, 0, buf, iters, 1u); break;
        case 1: hipLaunchKernelGGL(k_rate<1>, dim3(blocks), dim3(kThreads), 0, 0, buf, iters, 1u); break;
        case 2: hipLaunchKernelGGL(k_rate<2>, dim3(blocks), dim3(kThreads), 0, 0, buf, iters, 1u); break;
        case 3: hipLaunchKernelGGL(k_rate<3>, dim3(blocks), dim3(kThreads), 0, 0, buf, iters, 1u); break;
        default: hipLaunchKernelGGL(k_rate<4>, dim3(blocks), dim3(kThreads), 0, 0, buf, iters, 1u); break;
      }
      if (hipGetLastError() != hipSuccess || hipEventRecord(b, 0) != hipSuccess ||
          hipEventSynchronize(b) != hipSuccess)
        rc = -2;
      float ms = 0.0f;
      if (rc == 0 && hipEventElapsedTime(&ms, a, b) != hipSuccess) rc = -2;
      if (rc == 0 && rep > 0 && (best < 0.0f || ms < best)) best = ms;
    }
    // wavefront steps per SIMD: 8 waves x iters x chains
    if (rc == 0) out[form] = (double)best * 1e6 / (8.0 * iters * kChains);
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(buf);
  return rc;
}
