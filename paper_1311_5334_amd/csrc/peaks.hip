// peaks.hip -- measured rates of the units the tracking kernels are bound
// by, timed on the device itself: 32-bit integer VALU lane operations
// (24-bit multiply-adds, the operation of the counting test), FP32 FMA lane
// operations (non-packed), LDS bytes read with 128-bit reads, and HBM bytes
// moved by a streaming copy. The counting kernel's roofline fractions are
// quoted against these beside the rates derived from the chip's unit counts
// and clock.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "emt.h"

namespace {

constexpr int kPeakBlock = 256;
constexpr int kChains = 8;   // independent dependency chains per lane
constexpr int kUnroll = 16;  // operations per chain per loop trip

// Every lane runs kChains independent chains of a = a * m + c on the low
// 24 bits of a and m, one v_mad_u32_u24 each (written as that instruction:
// the compiler otherwise merges the steps into full 32-bit multiplies); the
// result feeds a store no input makes happen, so nothing is folded away.
__global__ void __launch_bounds__(kPeakBlock) k_peak_int(uint32_t *sink, uint32_t m24, uint32_t c,
                                                          int trips) {
    const uint32_t m = m24;
    uint32_t a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = threadIdx.x * 7u + (uint32_t)k + blockIdx.x;
    for (int t = 0; t < trips; ++t) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int k = 0; k < kChains; ++k)
                asm volatile("v_mad_u32_u24 %0, %0, %1, %2" : "+v"(a[k]) : "v"(m), "v"(c));
        }
    }
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) x ^= a[k];
    if (x == 0x9e3779b9u) sink[0] = x;
}

// The same with a = a * m + c in FP32 (one v_fma_f32 each).
__global__ void __launch_bounds__(kPeakBlock) k_peak_fma(float *sink, float m, float c, int trips) {
    float a[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) a[k] = (float)(threadIdx.x + k) * 1e-3f;
    for (int t = 0; t < trips; ++t) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
#pragma unroll
            for (int k = 0; k < kChains; ++k) a[k] = fmaf(a[k], m, c);
        }
    }
    float x = 0.0f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) x += a[k];
    if (x == 1234.5f) sink[0] = x;
}

// LDS: each lane reads 16 bytes at a time from a 32 KB array, 15 reads per
// trip at constant offsets from its own address (ds_read_b128 with an
// immediate offset), folding them into a running xor.
constexpr int kLdsWords = 2048;  // uint4 entries: 32 KB
__global__ void __launch_bounds__(kPeakBlock) k_peak_lds(uint32_t *sink, int trips) {
    __shared__ uint4 buf[kLdsWords];
    for (int i = threadIdx.x; i < kLdsWords; i += kPeakBlock)
        buf[i] = make_uint4(i, i * 3u, i * 5u, i * 7u);
    __syncthreads();
    uint4 acc = make_uint4(0, 0, 0, 0);
    const uint4 *p = buf + threadIdx.x;
    for (int t = 0; t < trips; ++t) {
#pragma unroll
        for (int u = 0; u < 15; ++u) {
            const uint4 v = p[u * 128];  // at most 255 + 14 * 128 < kLdsWords
            acc.x ^= v.x;
            acc.y ^= v.y;
            acc.z ^= v.z;
            acc.w ^= v.w;
        }
        p = buf + ((threadIdx.x + (uint32_t)t) & (kPeakBlock - 1));
    }
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x9e3779b9u) sink[0] = acc.x;
}

// HBM: a grid-stride copy of 16-byte words.
__global__ void __launch_bounds__(kPeakBlock) k_peak_copy(const uint4 *__restrict__ src,
                                                           uint4 *__restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * kPeakBlock;
    for (size_t i = (size_t)blockIdx.x * kPeakBlock + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

// Fastest of reps timed launches; returns milliseconds or a negative value
// on a HIP error.
template <typename F>
float best_ms(hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, F launch) {
    float best = 1e30f;
    launch();  // warm-up
    for (int r = 0; r < reps; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) return -1.0f;
        launch();
        if (hipEventRecord(e1, s) != hipSuccess) return -1.0f;
        if (hipEventSynchronize(e1) != hipSuccess) return -1.0f;
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0f;
        best = std::min(best, ms);
    }
    return hipGetLastError() == hipSuccess ? best : -1.0f;
}

}  // namespace

extern "C" int emt_measure_peaks(int32_t device, emt_peaks *out) {
    if (!out) return EMT_EINVAL;
    *out = emt_peaks{};
    int n_dev = 0;
    if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev)
        return EMT_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return EMT_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return EMT_EDEVICE;
    const size_t copy_words = (size_t)1 << 26;  // 1 GiB each way
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void *sink = nullptr, *src = nullptr, *dst = nullptr;
    int rc = EMT_EDEVICE;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess &&
        hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
        hipMalloc(&sink, 256) == hipSuccess &&
        hipMalloc(&src, copy_words * sizeof(uint4)) == hipSuccess &&
        hipMalloc(&dst, copy_words * sizeof(uint4)) == hipSuccess &&
        hipMemsetAsync(src, 1, copy_words * sizeof(uint4), s) == hipSuccess) {
        // eight workgroups of four waves per CU, several generations deep
        const uint32_t blocks = (uint32_t)prop.multiProcessorCount * 8u * 4u;
        const double lanes = (double)blocks * kPeakBlock;
        const int trips = 256;
        const double ops = lanes * trips * kUnroll * kChains;
        const float t_int = best_ms(s, e0, e1, 5, [&] {
            k_peak_int<<<blocks, kPeakBlock, 0, s>>>((uint32_t *)sink, 0x9u, 0x7u, trips);
        });
        const float t_fma = best_ms(s, e0, e1, 5, [&] {
            k_peak_fma<<<blocks, kPeakBlock, 0, s>>>((float *)sink, 0.999f, 1e-3f, trips);
        });
        // LDS: 32 KB a workgroup, four resident per CU
        const uint32_t lblocks = (uint32_t)prop.multiProcessorCount * 4u * 8u;
        const int ltrips = 512;
        const float t_lds = best_ms(s, e0, e1, 5, [&] {
            k_peak_lds<<<lblocks, kPeakBlock, 0, s>>>((uint32_t *)sink, ltrips);
        });
        const float t_copy = best_ms(s, e0, e1, 5, [&] {
            k_peak_copy<<<(uint32_t)prop.multiProcessorCount * 16u, kPeakBlock, 0, s>>>(
                (const uint4 *)src, (uint4 *)dst, copy_words);
        });
        if (t_int > 0 && t_fma > 0 && t_lds > 0 && t_copy > 0) {
            out->int_lane_ops = ops / (t_int * 1e-3);
            out->fp32_lane_ops = ops / (t_fma * 1e-3);
            out->lds_bytes = (double)lblocks * kPeakBlock * ltrips * 15.0 * 16.0 / (t_lds * 1e-3);
            out->hbm_copy_bytes = 2.0 * (double)copy_words * sizeof(uint4) / (t_copy * 1e-3);
            out->compute_units = (uint32_t)prop.multiProcessorCount;
            out->clock_khz = (uint32_t)prop.clockRate;
            rc = EMT_OK;
        }
    }
    if (src) (void)hipFree(src);
    if (dst) (void)hipFree(dst);
    if (sink) (void)hipFree(sink);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipStreamDestroy(s);
    (void)hipGetLastError();
    return rc;
}
