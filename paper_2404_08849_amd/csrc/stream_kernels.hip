// Streaming kernels: the HBM bandwidth a purely streaming kernel reaches on
// this device, the ceiling the stencil kernels' achieved bandwidth is read
// against.  Not a step of the dycore.
//
// Each lane moves four 16-byte words (dwordx4 loads and stores, consecutive
// lanes on consecutive words, so a wave touches 1 KiB contiguous per
// instruction); a work-group of 256 lanes covers 16 KiB, and the grid covers
// the buffer once.  Read mode folds the words it loads into one 8-byte value
// per work-group, stored at the start of dst, so the loads cannot be removed.
#include <hip/hip_runtime.h>

#include "mpdc_internal.h"

namespace mpdc {
namespace {

constexpr int kStreamThreads = 256;
constexpr int kStreamUnroll = 4;

enum { STREAM_READ = 0, STREAM_WRITE = 1, STREAM_COPY = 2 };

template <int MODE>
__global__ void __launch_bounds__(kStreamThreads) k_stream(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                          long n16) {
    const long base = (long)blockIdx.x * (kStreamThreads * kStreamUnroll) + threadIdx.x;
    uint4 v[kStreamUnroll];
    if constexpr (MODE != STREAM_WRITE) {
#pragma unroll
        for (int j = 0; j < kStreamUnroll; j++) {
            const long i = base + (long)j * kStreamThreads;
            v[j] = i < n16 ? src[i] : make_uint4(0u, 0u, 0u, 0u);
        }
    }
    if constexpr (MODE == STREAM_READ) {
        unsigned x = 0u;
#pragma unroll
        for (int j = 0; j < kStreamUnroll; j++) x ^= v[j].x ^ v[j].y ^ v[j].z ^ v[j].w;
        __shared__ unsigned red[kStreamThreads];
        red[threadIdx.x] = x;
        __syncthreads();
        for (int s = kStreamThreads / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] ^= red[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            uint2 *out = reinterpret_cast<uint2 *>(dst);
            out[blockIdx.x] = make_uint2(red[0], blockIdx.x);
        }
    } else {
#pragma unroll
        for (int j = 0; j < kStreamUnroll; j++) {
            const long i = base + (long)j * kStreamThreads;
            if (i < n16) {
                if constexpr (MODE == STREAM_WRITE)
                    dst[i] = make_uint4((unsigned)i, 0x3f800000u, (unsigned)(i >> 32), 0u);
                else
                    dst[i] = v[j];
            }
        }
    }
}

}  // namespace

hipError_t launch_stream(int mode, const void *src, void *dst, long n16, hipStream_t s) {
    const long per_block = (long)kStreamThreads * kStreamUnroll;
    const unsigned blocks = (unsigned)((n16 + per_block - 1) / per_block);
    const uint4 *in = static_cast<const uint4 *>(src);
    uint4 *out = static_cast<uint4 *>(dst);
    switch (mode) {
    case STREAM_READ: hipLaunchKernelGGL(k_stream<STREAM_READ>, dim3(blocks), dim3(kStreamThreads), 0, s, in, out, n16); break;
    case STREAM_WRITE: hipLaunchKernelGGL(k_stream<STREAM_WRITE>, dim3(blocks), dim3(kStreamThreads), 0, s, in, out, n16); break;
    case STREAM_COPY: hipLaunchKernelGGL(k_stream<STREAM_COPY>, dim3(blocks), dim3(kStreamThreads), 0, s, in, out, n16); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

long stream_blocks(long n16) {
    const long per_block = (long)kStreamThreads * kStreamUnroll;
    return (n16 + per_block - 1) / per_block;
}

}  // namespace mpdc
