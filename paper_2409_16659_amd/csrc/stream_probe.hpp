// stream_probe.hpp -- streaming bandwidth probes for gfx950: the rate that
// a single-pass kernel with the step kernel's access width reaches on a
// buffer of a given size (the practical ceiling for the step), and a kernel
// of exactly known traffic for scaling the memory counters.
//
// Every lane moves 16 bytes per access through raw buffer loads and stores
// (the widest vector access), kStreamUnroll independent accesses in flight
// per lane.  Two schedules:
//   chunked      workgroup b owns one contiguous range of the buffer and
//                walks it front to back (each workgroup one sequential
//                stream; the fastest schedule for HBM-sized buffers)
//   grid-stride  all lanes sweep the buffer together, lane t taking
//                elements t, t + T, t + 2T, ... (T = lanes in the grid)
// Modes:
//   read   load every byte of src once (XOR-folded; one conditional store
//          per lane keeps the loads alive and never fires in practice)
//   write  store a pattern over every byte of dst once
//   copy   dst <- src
// AUX is the buffer instructions' cache-policy operand (0: default,
// 2: non-temporal).  Elements past the end use an offset beyond the
// descriptor's size: loads return zero and stores are dropped.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlf {

enum StreamMode { kStreamRead = 0, kStreamWrite = 1, kStreamCopy = 2 };
constexpr int kStreamThreads = 256;
constexpr int kStreamUnroll = 4;
constexpr uint32_t kStreamPast = 0xfffffff0u;  // offset of an element past the end

typedef unsigned int sp_u32x4 __attribute__((ext_vector_type(4)));

__device__ inline __amdgpu_buffer_rsrc_t stream_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

// n16 = number of 16-byte elements (buffers of at most 4 GiB - 16 bytes);
// chunk = elements per workgroup for the chunked schedule, 0 for grid-stride.
template <int MODE, int AUX>
__global__ void __launch_bounds__(kStreamThreads)
stream_probe_kernel(const unsigned char* __restrict__ src, unsigned char* __restrict__ dst, uint32_t n16,
                    uint32_t chunk) {
  const uint32_t bytes = n16 * 16u;
  const __amdgpu_buffer_rsrc_t rs = stream_rsrc(src, bytes);
  const __amdgpu_buffer_rsrc_t rd = stream_rsrc(dst, bytes);
  uint64_t first, end, stride;
  if (chunk) {
    first = (uint64_t)blockIdx.x * chunk + threadIdx.x;
    end = (uint64_t)blockIdx.x * chunk + chunk;
    end = end < n16 ? end : n16;
    stride = kStreamThreads;
  } else {
    first = (uint64_t)blockIdx.x * kStreamThreads + threadIdx.x;
    end = n16;
    stride = (uint64_t)gridDim.x * kStreamThreads;
  }
  uint32_t acc = 0;
  for (uint64_t base = first; base < end; base += kStreamUnroll * stride) {
    sp_u32x4 v[kStreamUnroll];
    if constexpr (MODE != kStreamWrite) {
#pragma unroll
      for (int u = 0; u < kStreamUnroll; ++u) {
        const uint64_t e = base + u * stride;
        const uint32_t off = e < end ? (uint32_t)(e * 16u) : kStreamPast;
        v[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, AUX);
      }
    }
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
      const uint64_t e = base + u * stride;
      const uint32_t off = e < end ? (uint32_t)(e * 16u) : kStreamPast;
      if constexpr (MODE == kStreamRead) {
        acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
      } else if constexpr (MODE == kStreamWrite) {
        __builtin_amdgcn_raw_buffer_store_b128(sp_u32x4{off, off + 4u, off + 8u, off + 12u}, rd, (int)off, 0, AUX);
      } else {
        __builtin_amdgcn_raw_buffer_store_b128(v[u], rd, (int)off, 0, AUX);
      }
    }
  }
  if constexpr (MODE == kStreamRead) {
    if (acc == 0x9e3779b9u) __builtin_amdgcn_raw_buffer_store_b32(acc, rd, 0, 0, 0);
  }
}

}  // namespace mlf
