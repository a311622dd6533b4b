// probe.hip -- measurement kernels for the step kernel's roofline: how fast
// the chip serves random gathers from LDS (state bytes, combined-table
// entries, slot and predictor records) and from a plan image in global memory
// through the vector L1.  They do no simulation work; the benchmark times them
// on the stream it launches them on and turns the rates into ceilings.
#include <hip/hip_runtime.h>

#include <string>

#include "internal.h"

namespace {

constexpr uint32_t kProbeThreads = 256;
constexpr int kProbeStreams = 8;   // independent gathers in flight per lane

// Per-lane start addresses: a hash of the lane's global index.
__device__ __forceinline__ uint32_t probe_hash(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

template <int WIDTH>
__device__ __forceinline__ uint32_t lds_read(const uint8_t* buf, uint32_t a) {
  if constexpr (WIDTH == 1) {
    return buf[a];
  } else if constexpr (WIDTH == 4) {
    return *reinterpret_cast<const uint32_t*>(buf + a);
  } else {
    const uint4 v = *reinterpret_cast<const uint4*>(buf + a);
    return v.x ^ v.y ^ v.z ^ v.w;
  }
}

// Random gathers of WIDTH bytes from a 2^log2_bytes-byte LDS buffer, one per
// workgroup.  pattern 0: every lane reads a random aligned address; pattern
// 1: lane L of a wave reads bank-distinct words (address (4 L) mod 128 plus a
// random row), the conflict-free case the swizzled record layout aims at.
// Each iteration moves every address by a lane-independent random step (one
// three-input bitwise op), so consecutive gathers stay independent.
template <int WIDTH>
__global__ void __launch_bounds__(kProbeThreads) k_probe_lds(uint32_t log2_bytes, uint32_t pattern, uint32_t iters,
                                                            uint32_t* sink) {
  extern __shared__ __attribute__((aligned(16))) uint8_t buf[];
  const uint32_t bytes = 1u << log2_bytes;
  for (uint32_t i = threadIdx.x * 4u; i < bytes; i += kProbeThreads * 4u)
    *reinterpret_cast<uint32_t*>(buf + i) = probe_hash(i);
  __syncthreads();
  const uint32_t gid = blockIdx.x * kProbeThreads + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t amask = (bytes - 1u) & ~uint32_t(WIDTH - 1);
  const uint32_t rmask = pattern ? (bytes - 1u) & ~127u : amask;   // pattern 1: random 128-byte row
  uint32_t a[kProbeStreams];
#pragma unroll
  for (int k = 0; k < kProbeStreams; ++k) {
    const uint32_t h = probe_hash(gid * kProbeStreams + k) & amask;
    a[k] = pattern ? (h & rmask) | ((lane * uint32_t(WIDTH)) & 127u & amask) : h;
  }
  uint32_t acc = 0, step = probe_hash(blockIdx.x);
  for (uint32_t it = 0; it < iters; ++it) {
    step = step * 1664525u + 1013904223u;   // the same for every lane
    const uint32_t d = step & rmask;
#pragma unroll
    for (int k = 0; k < kProbeStreams; ++k) {
      acc += lds_read<WIDTH>(buf, a[k]);
      a[k] ^= d;                              // stays aligned, in range, bank-distinct under pattern 1
    }
  }
  if (acc == 0x9E3779B9u) sink[0] = gid;   // keeps the reads; practically never stores
}

// Gathers of WIDTH bytes (1 or 16) from a global buffer of 2^log2_bytes bytes
// through the vector L1 and L2: the path a plan image in global memory takes.
// pattern 0: every lane reads a random aligned address (16-byte records,
// one-byte table entries of scattered slots); pattern 1: lane L reads unit L
// of a random row of 64 WIDTH bytes, the coalesced read of a pass's slot
// records.  A buffer that fits the vector L1 gives the rate at which every
// read hits it.
template <int WIDTH>
__global__ void __launch_bounds__(kProbeThreads) k_probe_vmem(const uint8_t* __restrict__ img, uint32_t log2_bytes,
                                                             uint32_t pattern, uint32_t iters, uint32_t* sink) {
  const uint32_t gid = blockIdx.x * kProbeThreads + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u;
  constexpr uint32_t kRow = 64u * WIDTH;
  const uint32_t amask = ((1u << log2_bytes) - 1u) & ~uint32_t(WIDTH - 1);
  const uint32_t rmask = pattern ? amask & ~(kRow - 1u) : amask;   // pattern 1: random row
  uint32_t a[kProbeStreams];
#pragma unroll
  for (int k = 0; k < kProbeStreams; ++k) {
    const uint32_t h = probe_hash(gid * kProbeStreams + k) & amask;
    a[k] = pattern ? (h & rmask) | (lane * uint32_t(WIDTH)) : h;
  }
  uint32_t acc = 0, step = probe_hash(blockIdx.x);
  for (uint32_t it = 0; it < iters; ++it) {
    step = step * 1664525u + 1013904223u;
    const uint32_t d = step & rmask;
#pragma unroll
    for (int k = 0; k < kProbeStreams; ++k) {
      if constexpr (WIDTH == 16) {
        const uint4 v = *reinterpret_cast<const uint4*>(img + a[k]);
        acc += v.x ^ v.y ^ v.z ^ v.w;
      } else {
        acc += img[a[k]];
      }
      a[k] ^= d;                              // stays aligned and in range; a row stays a row
    }
  }
  if (acc == 0x9E3779B9u) sink[0] = gid;
}

pbn_status probe_fail(pbn_status code, const std::string& msg) {
  pbn::set_error(msg);
  return code;
}

}  // namespace

extern "C" pbn_status pbn_probe_lds_gather(uint32_t log2_bytes, uint32_t width, uint32_t pattern, uint32_t iters,
                                           uint32_t blocks, uint32_t* d_sink, void* stream) {
  pbn::clear_error();
  if (!d_sink) return probe_fail(PBN_EINVAL, "null argument");
  if (log2_bytes < 7 || log2_bytes > 16) return probe_fail(PBN_EINVAL, "LDS buffer must be 2^7 .. 2^16 bytes");
  if (width != 1 && width != 4 && width != 16) return probe_fail(PBN_EINVAL, "width must be 1, 4 or 16 bytes");
  if (pattern > 1 || blocks == 0) return probe_fail(PBN_EINVAL, "bad pattern or block count");
  const uint32_t lds = 1u << log2_bytes;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (width == 1)
    hipLaunchKernelGGL(k_probe_lds<1>, dim3(blocks), dim3(kProbeThreads), lds, s, log2_bytes, pattern, iters, d_sink);
  else if (width == 4)
    hipLaunchKernelGGL(k_probe_lds<4>, dim3(blocks), dim3(kProbeThreads), lds, s, log2_bytes, pattern, iters, d_sink);
  else
    hipLaunchKernelGGL(k_probe_lds<16>, dim3(blocks), dim3(kProbeThreads), lds, s, log2_bytes, pattern, iters, d_sink);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PBN_OK : probe_fail(PBN_EHIP, std::string("probe launch: ") + hipGetErrorString(e));
}

extern "C" pbn_status pbn_probe_vmem_gather(const void* d_buf, uint32_t log2_bytes, uint32_t width, uint32_t pattern,
                                            uint32_t iters, uint32_t blocks, uint32_t* d_sink, void* stream) {
  pbn::clear_error();
  if (!d_buf || !d_sink) return probe_fail(PBN_EINVAL, "null argument");
  if (log2_bytes < 4 || log2_bytes > 30 || blocks == 0) return probe_fail(PBN_EINVAL, "bad buffer size or block count");
  if (width != 1 && width != 16) return probe_fail(PBN_EINVAL, "width must be 1 or 16 bytes");
  if (pattern > 1) return probe_fail(PBN_EINVAL, "bad pattern");
  if (pattern == 1 && (1u << log2_bytes) < 64u * width)
    return probe_fail(PBN_EINVAL, "pattern 1 needs a buffer of at least one row (64 x width bytes)");
  if (width == 16)
    hipLaunchKernelGGL(k_probe_vmem<16>, dim3(blocks), dim3(kProbeThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const uint8_t*>(d_buf), log2_bytes, pattern, iters, d_sink);
  else
    hipLaunchKernelGGL(k_probe_vmem<1>, dim3(blocks), dim3(kProbeThreads), 0, static_cast<hipStream_t>(stream),
                       static_cast<const uint8_t*>(d_buf), log2_bytes, pattern, iters, d_sink);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? PBN_OK : probe_fail(PBN_EHIP, std::string("probe launch: ") + hipGetErrorString(e));
}
