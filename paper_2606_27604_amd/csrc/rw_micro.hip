// Issue-rate micro-benchmarks of the VALU instruction classes the walk uses
// (gfx950).  Each thread runs 8 independent dependency chains of one
// instruction so that throughput, not latency, limits the loop; the result is
// written out so nothing is eliminated.  Used by bench.py --micro to check the
// per-class issue costs that the ALU roofline weights (full-rate = 1 cycle per
// wave64 instruction per SIMD pass of 16 lanes; quarter-rate = 4).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rw_device.hpp"

namespace {

constexpr int kChains = 8;

enum Op : int {
  OP_FMA = 0,
  OP_MAD_U64 = 1,
  OP_XOR3 = 2,
  OP_LOG = 3,
  OP_SIN = 4,
  OP_RCP = 5,
  OP_SQRT = 6,
  OP_RSQ = 7,
  OP_MULHI = 8,
  OP_PHILOX = 9,
  OP_LOG_MIX = 10,  // four FMAs then one log per chain: a transcendental amid VALU work
  OP_COUNT = 11
};

template <int OP>
__global__ void __launch_bounds__(256) micro_kernel(int iters, uint32_t seed, uint32_t* out) {
  const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
  float f[kChains];
  uint32_t w[kChains];
  uint64_t q[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    f[c] = 1.0f + 1e-3f * float((tid + c) & 255);
    w[c] = tid * 2654435761u + c * 97u + seed;
    q[c] = w[c];
  }
  const rw::PhiloxKey ks = rw::philox_schedule(seed, seed ^ 0x55u);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      // one instruction per chain and iteration (values may degenerate; the
      // issue rate does not depend on them)
      if (OP == OP_FMA) f[c] = fmaf(f[c], 0.999f, 1e-3f);
      if (OP == OP_MAD_U64) {  // two products per chain (ping-pong keeps dst != src)
        const uint64_t t = uint64_t(uint32_t(q[c])) * 0xD2511F53u + q[c];
        q[c] = uint64_t(uint32_t(t)) * 0xCD9E8D57u + t;
      }
      if (OP == OP_XOR3) w[c] = rw::xor3(w[c], w[(c + 3) & (kChains - 1)], ks.k0);
      if (OP == OP_LOG) f[c] = __builtin_amdgcn_logf(f[c]);
      if (OP == OP_SIN) f[c] = __builtin_amdgcn_sinf(f[c]);
      if (OP == OP_RCP) f[c] = __builtin_amdgcn_rcpf(f[c]);
      if (OP == OP_SQRT) f[c] = __builtin_amdgcn_sqrtf(f[c]);
      if (OP == OP_RSQ) f[c] = __builtin_amdgcn_rsqf(f[c]);
      if (OP == OP_MULHI) w[c] = __umulhi(w[c], 0xCD9E8D57u);
      if (OP == OP_LOG_MIX)
        f[c] = __builtin_amdgcn_logf(
            fmaf(fmaf(fmaf(fmaf(f[c], 0.999f, 1e-3f), 0.999f, 1e-3f), 0.999f, 1e-3f), 0.999f, 2.0f));
      if (OP == OP_PHILOX && c == 0) {
        const uint4 r = rw::philox(w[0], w[1], w[2], w[3], ks);
        w[0] = r.x; w[1] = r.y; w[2] = r.z; w[3] = r.w;
      }
    }
  }
  uint32_t acc = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) acc += w[c] ^ __float_as_uint(f[c]) ^ uint32_t(q[c] >> 17);
  out[tid] = acc;
}

}  // namespace

extern "C" {

// Runs `op` with grid x 256 threads, `iters` iterations of 8 chains each (two
// products per chain for the 64-bit multiply-add, one block for Philox); returns
// milliseconds (hipEvent) or a negative value on error.  out: device uint32
// [grid * 256].
float rw_micro_run(int op, int grid, int iters, uint32_t* out) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0f;
  hipEventRecord(e0, nullptr);
  switch (op) {
#define MICRO_CASE(X) \
    case X: hipLaunchKernelGGL(micro_kernel<X>, dim3(grid), dim3(256), 0, nullptr, iters, 1u, out); break;
    MICRO_CASE(OP_FMA)
    MICRO_CASE(OP_MAD_U64)
    MICRO_CASE(OP_XOR3)
    MICRO_CASE(OP_LOG)
    MICRO_CASE(OP_SIN)
    MICRO_CASE(OP_RCP)
    MICRO_CASE(OP_SQRT)
    MICRO_CASE(OP_RSQ)
    MICRO_CASE(OP_MULHI)
    MICRO_CASE(OP_PHILOX)
    MICRO_CASE(OP_LOG_MIX)
#undef MICRO_CASE
    default: return -2.0f;
  }
  hipEventRecord(e1, nullptr);
  if (hipEventSynchronize(e1) != hipSuccess) return -3.0f;
  float ms = 0.0f;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return ms;
}

int rw_micro_op_count(void) { return OP_COUNT; }
}
