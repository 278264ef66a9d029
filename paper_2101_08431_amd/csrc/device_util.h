// Block- and wave-level building blocks shared by the HIP kernels.  Every
// reduction here runs in a fixed order, so results do not depend on block
// scheduling.
#pragma once
#include <hip/hip_runtime.h>

#include "nmf_internal.h"

namespace nmfk {

// Counts the block in; returns true in the block that arrives last.  The
// counter wraps to zero at `expected` in the same atomic (atomicInc), so it is
// ready for the next launch without another write.  All threads of the block
// call it.
__device__ __forceinline__ bool last_arrival(unsigned *cnt, unsigned expected, unsigned *flag_lds) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned old = atomicInc(cnt, expected - 1u);
        *flag_lds = (old == expected - 1u) ? 1u : 0u;
    }
    __syncthreads();
    const bool last = (*flag_lds != 0u);
    if (last) __threadfence();
    return last;
}

// One butterfly step: lanes that differ in bit H swap halves of v[0..2H) and
// keep the sum of the half named by their bit.
template <int H, int N, class T>
__device__ __forceinline__ void transpose_step(T (&v)[N], int lane) {
    static_assert(2 * H <= N, "step wider than the vector");
    const bool up = (lane & H) != 0;
#pragma unroll
    for (int q = 0; q < H; ++q) {
        const double send = up ? v[q] : v[q + H];
        const double keep = up ? v[q + H] : v[q];
        v[q] = keep + __shfl_xor(send, H, 64);
    }
}

// Lane l of the wave ends up with the sum over the 64 lanes of v[l].
template <class T>
__device__ __forceinline__ T wave_transpose_reduce(T (&v)[YVALS], int lane) {
    transpose_step<32>(v, lane);
    transpose_step<16>(v, lane);
    transpose_step<8>(v, lane);
    transpose_step<4>(v, lane);
    transpose_step<2>(v, lane);
    transpose_step<1>(v, lane);
    return v[0];
}

// The same for 32 values: lanes l and l + 32 end up with the sum over the 64
// lanes of v[l mod 32] (31 exchanges within each half of the wave and one
// across, instead of 63).
template <class T>
__device__ __forceinline__ T wave_transpose_reduce32(T (&v)[32], int lane) {
    transpose_step<16>(v, lane);
    transpose_step<8>(v, lane);
    transpose_step<4>(v, lane);
    transpose_step<2>(v, lane);
    transpose_step<1>(v, lane);
    return v[0] + __shfl_xor((double)v[0], 32, 64);
}

// Fixed-order sum of `cnt` records of `len` doubles (stride `len`) into
// out[0..len) (LDS), using the whole block: thread (q, g) sums the records
// g, g + G, g + 2G, ... of entry q (G = blockDim / len groups), then the G
// group sums are added in order.  `scratch` holds blockDim doubles of LDS.
// Ends with a barrier.  len <= blockDim.  It is split in two so that a kernel
// can issue the loads (records_partial: thread tid of nthr threads returns its
// group sum, no barrier) together with its other loads and add them up later
// (records_finish).  Records past the end count as zero, so the order of the
// real ones is unchanged.
__device__ __forceinline__ double records_partial(const double *src, int cnt, int len, int tid, int nthr) {
    const int G = nthr / len;
    if (G <= 0) return 0.0;   // len > nthr: not a supported call
    const int q = tid % len, g = tid / len;
    // threads past the G groups, and records past the end, load record 0 or
    // cnt - 1 and drop it: 16 loads in flight per step, no branch between
    // them (one step covers 16 G records)
    constexpr int D = 16;
    const int gc = g < G ? g : 0;
    double acc = 0.0;
    for (int t = gc; t < cnt; t += D * G) {
        double a[D];
#pragma unroll
        for (int u = 0; u < D; ++u) a[u] = src[(size_t)min(t + u * G, cnt - 1) * len + q];
#pragma unroll
        for (int u = 0; u < D; ++u) acc += t + u * G < cnt ? a[u] : 0.0;
    }
    return g < G ? acc : 0.0;
}

// Second half of reduce_records: the partials of threads [base, base + nthr)
// go through scratch[base ..) and thread base + q < base + len adds its entry's
// G group sums in order into out[q].  Ends with a barrier.
__device__ __forceinline__ void records_finish(double acc, int len, int base, int nthr, double *out,
                                               double *scratch) {
    const int G = nthr / len;
    scratch[threadIdx.x] = acc;
    __syncthreads();
    const int tid = (int)threadIdx.x - base;
    if (tid >= 0 && tid < len) {
        double s = 0.0;
        for (int gg = 0; gg < G; ++gg) s += scratch[base + gg * len + tid];
        out[tid] = s;
    }
    __syncthreads();
}

__device__ __forceinline__ void reduce_records(const double *src, int cnt, int len, double *out,
                                               double *scratch) {
    const double acc = records_partial(src, cnt, len, (int)threadIdx.x, (int)blockDim.x);
    records_finish(acc, len, 0, (int)blockDim.x, out, scratch);
}

// Sums V values per thread over a block of NTHR threads: wave transpose-reduce
// passes of 64 values, then the NTHR/64 waves in order.  Thread q < V ends up
// writing the block sum of value q to out[q] (global).  lds holds NTHR doubles.
// All threads call it.
template <int V>
__device__ __forceinline__ void block_reduce_to(const double (&vals)[V], double *out, double *lds) {
    constexpr int NPASS = (V + YVALS - 1) / YVALS;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
        double v[YVALS];
#pragma unroll
        for (int q = 0; q < YVALS; ++q) v[q] = (pass * YVALS + q < V) ? vals[(pass * YVALS + q) % V] : 0.0;
        lds[w * YVALS + lane] = wave_transpose_reduce(v, lane);
        __syncthreads();
        const int idx = pass * YVALS + (int)threadIdx.x;
        if ((int)threadIdx.x < YVALS && idx < V) {
            double sum = lds[threadIdx.x];
            for (int ww = 1; ww < (int)blockDim.x / 64; ++ww) sum += lds[ww * YVALS + threadIdx.x];
            out[idx] = sum;
        }
        __syncthreads();
    }
}

// Wave minimum (fixed butterfly order).
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int h = 32; h >= 1; h >>= 1) {
        const double o = __shfl_xor(v, h, 64);
        v = o < v ? o : v;
    }
    return v;
}

}  // namespace nmfk
