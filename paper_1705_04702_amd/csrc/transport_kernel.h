// transport_kernel.h -- the persistent packet-queue transport kernel.
//
// One lane holds one photon packet in registers (the packet state is a
// structure of arrays across the 64 lanes of a wave).  Waves are persistent:
// each loops until the global work queue is drained, the analogue of the
// thread pool that keeps taking the next task index with an atomic increment
// (Section 5.2, Parallel class, Fig. 6).  Work is taken in chunks of packets
// with one atomic per wave; within a wave
//   * dead lanes are refilled from the wave's chunk, ranked by mbcnt over the
//     ballot of dead lanes (compaction of live packets);
//   * all marching lanes advance their ray march one cell per iteration in
//     lock step, whatever the march is for (propagation with deposits,
//     interaction search or peel-off optical depth);
//   * once at least `threshold` lanes have finished their march (ballot), the
//     finished lanes process their event and start their next march.
// Per-wavelength optics and the instrument frames are staged in LDS.  The
// absorbed luminosity goes to the FP64 (wavelength, cell) table through
// hardware FP64 atomic adds, the GPU form of the lock-free addition of
// Section 5.2; peel-offs go to the images through hardware float atomics.
#pragma once

#include <hip/hip_runtime.h>

#define MCRT_HD __device__ __forceinline__
#include "transport_core.h"
#include "internal.h"

namespace mcrt {

struct DevSink {
    __device__ __forceinline__ void deposit(double *p, double v)
    {
        if (v != 0.0) unsafeAtomicAdd(p, v);
    }
    __device__ __forceinline__ void pixel(float *p, float v) { unsafeAtomicAdd(p, v); }
    __device__ __forceinline__ void pixel(double *p, double v) { unsafeAtomicAdd(p, v); }
};

__device__ __forceinline__ uint32_t lanes_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ double wave_sum(double x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

template <typename Real, typename ImgT, int G>
__global__ void __launch_bounds__(kBlock) transport_kernel(TransportArgs<Real, ImgT, G> a)
{
    __shared__ Optics<Real> s_opt[kMaxLdsLambda];
    __shared__ InsDesc<Real> s_ins[kMaxIns];
    View<Real, ImgT, G> v = a.view;
    if (v.n_lambda <= kMaxLdsLambda) {
        for (int i = threadIdx.x; i < v.n_lambda; i += blockDim.x) s_opt[i] = a.optics[i];
        v.optics = s_opt;
    } else {
        v.optics = a.optics;
    }
    for (int i = threadIdx.x; i < v.n_ins; i += blockDim.x) s_ins[i] = a.ins[i];
    v.ins = s_ins;
    __syncthreads();

    DevSink sink;
    const int lane = __lane_id();
    Lane<Real> ln;
    ln.mode = kDead;
    ln.marching = false;
    Tally ty = {};
    uint64_t cur = 0, end = 0;
    bool exhausted = false;

    for (;;) {
        // refill dead lanes from the wave's chunk (one atomic per chunk); a
        // refilled lane only launches here, its events run below
        bool launched = false;
        for (;;) {
            unsigned long long dead = __ballot(ln.mode == kDead && !launched);
            if (dead == 0 || exhausted) break;
            if (cur >= end) {
                unsigned long long c = 0;
                if (lane == 0) c = atomicAdd(a.counter, 1ull);
                c = __shfl(c, 0, 64);
                uint64_t base = (uint64_t)c * a.chunk;
                if (base >= a.total) {
                    exhausted = true;
                    break;
                }
                cur = base;
                end = base + a.chunk < a.total ? base + a.chunk : a.total;
                continue;
            }
            uint64_t avail = end - cur;
            uint32_t rank = lanes_below(dead);
            if (ln.mode == kDead && !launched && (uint64_t)rank < avail) {
                uint64_t P = cur + rank;
                uint32_t lam = (uint32_t)(P / a.count);
                uint32_t id = (uint32_t)(a.first_id + P % a.count);
                launch(v, ln, ty, lam, id, (uint32_t)P);
                launched = true;
            }
            uint64_t ndead = (uint64_t)__popcll(dead);
            cur += ndead < avail ? ndead : avail;
        }
        // events of the lanes whose march ended (or that just launched)
        if (!ln.marching && ln.mode != kDead) settle(v, ln, ty, sink);
        if (__ballot(ln.mode != kDead) == 0) {
            if (exhausted) break;
            continue;
        }

        // march: every marching lane advances one cell per iteration
        for (;;) {
            if (ln.marching) march_step(v, ln, ty, sink);
            unsigned long long waiting = __ballot(!ln.marching && (ln.mode != kDead || !exhausted));
            unsigned long long active = __ballot(ln.marching);
            if (active == 0 || __popcll(waiting) >= a.threshold) break;
        }
    }

    double e0 = wave_sum(ty.emitted), e1 = wave_sum(ty.absorbed);
    double e2 = wave_sum(ty.escaped), e3 = wave_sum(ty.truncated);
    unsigned long long s[kNumStats] = {ty.packets, ty.events, ty.prop_cells, ty.locate_cells,
                                       ty.peel_cells, ty.peel_adds, ty.peel_dropped, ty.capped,
                                       ty.guard};
#pragma unroll
    for (int i = 0; i < kNumStats; ++i) s[i] = wave_sum_u64(s[i]);
    if (lane == 0) {
        unsafeAtomicAdd(&a.energy[0], e0);
        unsafeAtomicAdd(&a.energy[1], e1);
        unsafeAtomicAdd(&a.energy[2], e2);
        unsafeAtomicAdd(&a.energy[3], e3);
#pragma unroll
        for (int i = 0; i < kNumStats; ++i)
            if (s[i]) atomicAdd(&a.stats[i], s[i]);
    }
}

// Copies a wave-uniform struct through readfirstlane, so the compiler keeps
// it in scalar registers.
template <typename T> __device__ __forceinline__ T uniform_copy(const T &src)
{
    static_assert(sizeof(T) % 4 == 0, "word-sized struct expected");
    T dst;
    const int *s = reinterpret_cast<const int *>(&src);
    int *d = reinterpret_cast<int *>(&dst);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = __builtin_amdgcn_readfirstlane(s[i]);
    return dst;
}

template <typename Real, typename ImgT, int G>
__device__ __forceinline__ void flush_tally(Tally &ty, double *energy, unsigned long long *stats, int lane)
{
    double e0 = wave_sum(ty.emitted), e1 = wave_sum(ty.absorbed);
    double e2 = wave_sum(ty.escaped), e3 = wave_sum(ty.truncated);
    unsigned long long s[kNumStats] = {ty.packets, ty.events, ty.prop_cells, ty.locate_cells,
                                       ty.peel_cells, ty.peel_adds, ty.peel_dropped, ty.capped,
                                       ty.guard};
#pragma unroll
    for (int i = 0; i < kNumStats; ++i) s[i] = wave_sum_u64(s[i]);
    if (lane == 0) {
        unsafeAtomicAdd(&energy[0], e0);
        unsafeAtomicAdd(&energy[1], e1);
        unsafeAtomicAdd(&energy[2], e2);
        unsafeAtomicAdd(&energy[3], e3);
#pragma unroll
        for (int i = 0; i < kNumStats; ++i)
            if (s[i]) atomicAdd(&stats[i], s[i]);
    }
    ty = Tally{};
}

// Batched launch over many Cartesian models (the many-small-models use case
// of Section 3.1 run as one persistent launch).  The queue is a list of chunks
// that never straddle models; a wave works on one model at a time, so the
// model's parameters are wave-uniform, and drains its lanes before it
// switches to a chunk of another model (tallies are flushed at the switch).
// The model index is the fourth word of every packet's Philox counter.
template <typename Real, typename ImgT>
__global__ void __launch_bounds__(kBlock) batch_transport_kernel(BatchArgs<Real, ImgT> a)
{
    DevSink sink;
    const int lane = __lane_id();
    Lane<Real> ln;
    ln.mode = kDead;
    ln.marching = false;
    Tally ty = {};
    int cur_model = -1, pend_model = -1;
    View<Real, ImgT, 0> v{};
    uint64_t count = 1, first_id = 0;
    uint64_t cur = 0, end = 0, pend_cur = 0, pend_end = 0;
    bool exhausted = false;

    for (;;) {
        bool launched = false;
        for (;;) {
            unsigned long long dead = __ballot(ln.mode == kDead && !launched);
            if (dead == 0 || exhausted) break;
            if (cur >= end) {
                if (pend_model < 0) {
                    unsigned long long c = 0;
                    if (lane == 0) c = atomicAdd(a.counter, 1ull);
                    c = __shfl(c, 0, 64);
                    if (c >= a.total_chunks) {
                        exhausted = true;
                        break;
                    }
                    int lo = 0, hi = a.n_models - 1; // last model with chunk0 <= c
                    while (lo < hi) {
                        int mid = (lo + hi + 1) >> 1;
                        if (a.models[mid].chunk0 <= c) lo = mid;
                        else hi = mid - 1;
                    }
                    pend_model = __builtin_amdgcn_readfirstlane(lo);
                    const ModelDesc<Real, ImgT> &m = a.models[pend_model];
                    pend_cur = (c - m.chunk0) * a.chunk;
                    pend_end = pend_cur + a.chunk < m.total ? pend_cur + a.chunk : m.total;
                }
                if (pend_model != cur_model) {
                    if (__ballot(ln.mode != kDead) != 0) break; // drain before switching
                    if (cur_model >= 0)
                        flush_tally<Real, ImgT, 0>(ty, a.models[cur_model].energy, a.models[cur_model].stats, lane);
                    cur_model = pend_model;
                    const ModelDesc<Real, ImgT> &m = a.models[cur_model];
                    v = uniform_copy(m.view);
                    v.optics = m.optics;
                    v.ins = m.ins;
                    count = m.count;
                    first_id = m.first_id;
                }
                cur = pend_cur;
                end = pend_end;
                pend_model = -1;
                continue;
            }
            uint64_t avail = end - cur;
            uint32_t rank = lanes_below(dead);
            if (ln.mode == kDead && !launched && (uint64_t)rank < avail) {
                uint64_t P = cur + rank;
                launch(v, ln, ty, (uint32_t)(P / count), (uint32_t)(first_id + P % count), (uint32_t)P);
                launched = true;
            }
            uint64_t ndead = (uint64_t)__popcll(dead);
            cur += ndead < avail ? ndead : avail;
        }
        if (!ln.marching && ln.mode != kDead) settle(v, ln, ty, sink);
        if (__ballot(ln.mode != kDead) == 0) {
            if (exhausted) break;
            continue;
        }
        for (;;) {
            if (ln.marching) march_step(v, ln, ty, sink);
            unsigned long long waiting = __ballot(!ln.marching && (ln.mode != kDead || !exhausted));
            unsigned long long active = __ballot(ln.marching);
            if (active == 0 || __popcll(waiting) >= a.threshold) break;
        }
    }
    if (cur_model >= 0) flush_tally<Real, ImgT, 0>(ty, a.models[cur_model].energy, a.models[cur_model].stats, lane);
}

template <typename Real, typename ImgT>
hipError_t launch_batch_impl(const BatchArgs<Real, ImgT> &a, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL((batch_transport_kernel<Real, ImgT>), dim3(grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

template <typename Real, typename ImgT, int G>
hipError_t launch_transport_impl(const TransportArgs<Real, ImgT, G> &a, int grid, hipStream_t stream)
{
    hipLaunchKernelGGL((transport_kernel<Real, ImgT, G>), dim3(grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

} // namespace mcrt
