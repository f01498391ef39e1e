// Gather probe: the bandwidth the memory hierarchy gives 16-byte gathers,
// the access the consistency kernels make (one bilinear cell per view and
// plane), measured from a buffer sized to live in one level -- an XCD's L2,
// the Infinity Cache, or HBM.  Not part of the method: it supplies the
// measured peaks the forward kernel's gathers are compared with.
//
// Each lane issues `iters` 16-byte loads at offsets from a counter-based
// 32-bit integer hash of (lane, iteration) (two multiplies and three
// xor-shifts, a few VALU per load so that the loads, not the index
// arithmetic, bound the probe), masked to the power-of-two buffer:
//   pattern 0  every lane its own random 16-byte element (a wave touches 64
//              cache lines: the L1 -> L2 request rate bounds it);
//   pattern 1  a wave reads one random 1 KiB block, lane i its i-th 16 bytes
//              (a wave touches 8 or 16 lines: the L2 data path bounds it).
// Four loads are kept in flight per lane; the sum of what was read goes to
// out_dev[global thread] so that no load is dead.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ecc.h"
#include "../../include/ecc_probe.h"
#include "ecc_internal.hpp"

namespace {

__device__ __forceinline__ uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <int PATTERN>
__global__ __launch_bounds__(256) void gather_probe_kernel(const float4 *__restrict__ buf, uint32_t elem_mask,
                                                           int iters, float *__restrict__ out) {
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = gtid >> 6;
    const uint32_t block_mask = elem_mask >> 6;  // 1 KiB blocks of 64 elements
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int i = 0; i < iters; i += 4) {
        float4 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t e;
            if (PATTERN == 0)
                e = hash32(gtid * 4096u + (uint32_t)(i + j)) & elem_mask;
            else
                e = ((hash32(wave * 4096u + (uint32_t)(i + j)) & block_mask) << 6) | lane;
            v[j] = buf[e];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            acc.x += v[j].x;
            acc.y += v[j].y;
            acc.z += v[j].z;
            acc.w += v[j].w;
        }
    }
    out[gtid] = acc.x + acc.y + acc.z + acc.w;
}

}  // namespace

extern "C" {

ecc_status ecc_probe_gather(const void *buf_dev, uint64_t bytes, int32_t pattern, int32_t iters, int32_t n_blocks,
                            float *out_dev, void *stream) {
    if (!buf_dev || !out_dev) return ecc::set_error(ECC_E_ARG, "null argument");
    if (bytes < 1024 || bytes > (1ull << 36) || (bytes & (bytes - 1)))
        return ecc::set_error(ECC_E_ARG, "buffer must be a power of two between 1 KiB and 64 GiB bytes");
    if (pattern != 0 && pattern != 1) return ecc::set_error(ECC_E_ARG, "unknown pattern %d", pattern);
    if (iters < 4 || iters > 4096 || iters % 4) return ecc::set_error(ECC_E_ARG, "iters must be a multiple of 4 in [4, 4096]");
    if (n_blocks < 1 || n_blocks > (1 << 20)) return ecc::set_error(ECC_E_ARG, "n_blocks out of range");
    const uint32_t elem_mask = (uint32_t)(bytes / 16 - 1);
    hipStream_t s = (hipStream_t)stream;
    if (pattern == 0)
        hipLaunchKernelGGL(gather_probe_kernel<0>, dim3(n_blocks), dim3(256), 0, s, (const float4 *)buf_dev, elem_mask,
                           iters, out_dev);
    else
        hipLaunchKernelGGL(gather_probe_kernel<1>, dim3(n_blocks), dim3(256), 0, s, (const float4 *)buf_dev, elem_mask,
                           iters, out_dev);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return ecc::set_error(ECC_E_HIP, "gather probe launch failed: %s", hipGetErrorString(e));
    return ECC_OK;
}

}  // extern "C"
