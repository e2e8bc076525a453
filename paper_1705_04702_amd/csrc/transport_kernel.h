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
//   * all marching lanes advance their ray march together, a fixed number of
//     cells per iteration (the geometric steps first, then their density
//     loads in flight together), whatever the march is for (propagation with
//     deposits, interaction search or peel-off optical depth);
//   * once at least `threshold` lanes have finished their march (ballot), the
//     finished lanes process their event and start their next march.
// Per-wavelength optics and the instrument frames are staged in LDS.  The
// absorbed luminosity goes to the FP64 (wavelength, cell) table through
// hardware FP64 atomic adds, the GPU form of the lock-free addition of
// Section 5.2 (issued transposed through LDS, see DevSink); peel-offs go to
// the images through hardware float atomics.
#pragma once

#include <hip/hip_runtime.h>

#define MCRT_HD __device__ __forceinline__
#include "transport_core.h"
#include "internal.h"
#include "proposal.h"

namespace mcrt {

// TRK > 0 (FP32 kernels): deposits go through a per-wave LDS tile of TRK
// slots per lane and are issued transposed -- one atomic instruction carries
// the slots of 64/TRK rays, a ray's slots in consecutive lanes, so the cells
// of one ray that share a line of the table travel as one L2 request (the L2
// retires FP64 atomics per 64-byte line request: ~1.8e11/s for 8 lanes on one
// line against ~2.4e10/s for 64 scattered lanes).  The deposits of a ray's
// open run -- its latest cells that share one line -- are held back while
// the propagation march goes on, so a run that spans two march iterations
// still goes out as one request (at most TRK - K slots are held: K new
// deposits per iteration always fit; TRK == K holds nothing).  Without held
// runs (HOLD false) a tile of TRK >= 2 K slots lets the wave skip the flush
// of every other iteration (see must_flush).  A slot holds the cell (u32) and
// the FP32 absorbed luminosity, which converts to FP64 exactly.
template <bool LEARN, bool HIST, int TRK = 0, int K = 0, bool HOLD = true> struct DevSink {
    static constexpr bool kLearn = LEARN, kHist = HIST;
    static constexpr int kPitch = 64 + (TRK > 0 ? 64 / TRK : 0); // slot-major rows, padded
    static constexpr bool kHold = HOLD && TRK > K;
    static_assert(TRK == 0 || (64 % TRK == 0 && TRK <= 16 && TRK >= K), "slot tile");
    uint32_t *sc = nullptr; // this lane's column of the wave's slot tiles
    float *sv = nullptr;
    int np = 0;        // slots in use
    int base = 0;      // ring position of the first slot in use (kHold)
    int run = 0;       // first slot (from base) of the open run
    uint32_t rl = ~0u; // table line of the open run
    __device__ __forceinline__ void deposit(double *table, long long slab, int cell, double v)
    {
        if constexpr (TRK > 0) {
            if (v != 0.0) {
                int slot = np;
                if constexpr (kHold) {
                    const uint32_t line = (uint32_t)cell >> 3;
                    if (line != rl) {
                        rl = line;
                        run = np;
                    }
                    slot = (base + np) & (TRK - 1);
                }
                sc[slot * kPitch] = (uint32_t)cell;
                sv[slot * kPitch] = (float)v;
                ++np;
            }
        } else {
            if (v != 0.0) unsafeAtomicAdd(table + slab + cell, v);
        }
    }
    // True when some lane of the wave could overflow its slots in the next
    // march iteration (K more deposits), so the wave must flush now.
    __device__ __forceinline__ bool must_flush() const { return __ballot(np > TRK - K) != 0; }
    // Issues the slots of closed runs; `hold` keeps the open run for the next
    // iteration (the lane's propagation march goes on).  Every lane posts one
    // word for its ray (wavelength, ring base, slots to issue), laid out so
    // that an issuing lane reads the words of all its rays with 128-bit loads;
    // the slots are read four rays at a time, so a flush waits on a few LDS
    // round trips.  table: the wave's table (uniform).  Whole wave active.
    __device__ __forceinline__ void flush(int lane, bool hold, int lam, double *table, long long n_store,
                                          const uint32_t *tile_c, const float *tile_v, uint32_t *wave_word)
    {
        if constexpr (TRK > 0) {
            constexpr int R = 64 / TRK;
            int keep = 0;
            if constexpr (kHold) {
                keep = hold ? np - run : 0;
                keep = keep < TRK - K ? keep : TRK - K;
            }
            const int lim = np - keep;
            // lam < 2^20 (the medium's limit), base < 16, lim <= 16
            wave_word[(lane % R) * TRK + lane / R] = ((uint32_t)lam << 9) | ((uint32_t)base << 5) | (uint32_t)lim;
            wave_lds_sync();
            const int s = lane % TRK, q = lane / TRK;
            constexpr int GW = TRK < 4 ? TRK : 4; // rays per group
#pragma unroll
            for (int g = 0; g < TRK / GW; ++g) {
                uint32_t w[GW];
                if constexpr (GW == 4) {
                    const uint4 x = reinterpret_cast<const uint4 *>(wave_word + q * TRK)[g];
                    w[0] = x.x;
                    w[1] = x.y;
                    w[2] = x.z;
                    w[3] = x.w;
                } else {
#pragma unroll
                    for (int i = 0; i < GW; ++i) w[i] = wave_word[q * TRK + GW * g + i];
                }
                uint32_t c[GW];
                float a[GW];
#pragma unroll
                for (int i = 0; i < GW; ++i) {
                    const int ray = R * (GW * g + i) + q;
                    const int slot = kHold ? (int)((((w[i] >> 5) & 15u) + (uint32_t)s) & (TRK - 1)) : s;
                    c[i] = tile_c[slot * kPitch + ray];
                    a[i] = tile_v[slot * kPitch + ray];
                }
#pragma unroll
                for (int i = 0; i < GW; ++i) {
                    if ((uint32_t)s < (w[i] & 31u)) {
                        double *p = table + ((long long)(w[i] >> 9) * n_store + c[i]);
                        __builtin_amdgcn_global_atomic_fadd_f64((__attribute__((address_space(1))) double *)p,
                                                                (double)a[i]);
                    }
                }
            }
            wave_lds_sync();
            if constexpr (kHold) {
                base = (base + lim) & (TRK - 1);
                run = 0;
            }
            np = keep;
        }
    }
    // Pixel adds are held in the lane (one pending add) and combined across
    // the wave at the next uniform point (flush_pixels); a second add before
    // that goes out directly.
    template <typename Real, typename T>
    __device__ __forceinline__ void pixel(Lane<Real> &ln, T *images, long long idx, T v)
    {
        if (ln.pix >= 0) unsafeAtomicAdd(images + ln.pix, (T)ln.pval);
        ln.pix = idx;
        ln.pval = (Real)v;
    }
};

// Second level of the pixel accumulation: one pixel per wave whose combined
// adds are summed in FP64 across flushes and added to the image once that
// pixel stops being the wave's combined pixel, and when the wave ends (or
// leaves the model's images).  The carry lives in a per-wave LDS slot (no
// registers held across the event loop): every lane reads it, lane 0 writes
// it; one wave's LDS operations complete in order.
struct PixelCarry {
    long long key; // image element, -1 when empty
    double val;
};

__device__ __forceinline__ void carry_init(PixelCarry *c, int lane)
{
    if (lane == 0) {
        c->key = -1;
        c->val = 0.0;
    }
}

template <typename ImgT> __device__ __forceinline__ void flush_carry(PixelCarry *c, ImgT *images, int lane)
{
    const long long key = c->key;
    const double val = c->val;
    if (key >= 0 && lane == 0) unsafeAtomicAdd(images + key, (ImgT)val);
    carry_init(c, lane);
}

// Wave-level combine of the pending pixel adds: the lanes whose pixel equals
// the first pending lane's pixel are summed across the wave (a point
// source's emission peel-offs all land in one pixel per wavelength) and
// join the wave's carry; the other lanes add their own.  Whole wave active.
template <typename Real, typename ImgT>
__device__ __forceinline__ void flush_pixels(Lane<Real> &ln, ImgT *images, int lane, PixelCarry *c)
{
    const unsigned long long m = __ballot(ln.pix >= 0);
    if (m == 0) return;
    const int leader = __ffsll((long long)m) - 1;
    const long long key = __shfl(ln.pix, leader, 64);
    const bool same = ln.pix == key;
    ImgT s = same ? (ImgT)ln.pval : (ImgT)0;
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    const long long ckey = c->key;
    const double cval = c->val;
    if (ckey >= 0 && ckey != key && lane == leader) unsafeAtomicAdd(images + ckey, (ImgT)cval);
    if (lane == leader) {
        c->key = key;
        c->val = (ckey == key ? cval : 0.0) + (double)s;
    }
    if (ln.pix >= 0 && !same) unsafeAtomicAdd(images + ln.pix, (ImgT)ln.pval);
    ln.pix = -1;
}

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

// Learned proposal, FP32: the lanes waiting for a direction are ranked
// (mbcnt over the ballot) and evaluated 16 at a time on the matrix cores;
// their features go through a per-wave LDS tile into the B operand, the 40
// outputs per sample come back through a second tile.  Must be called with
// the whole wave active.
template <typename ImgT, int G>
__device__ __forceinline__ void resolve_wave(const View<float, ImgT, G> &v, Lane<float> &ln, Tally &ty,
                                             const bf16x4 *Wf, const float *bias, uint16_t *feat, float *stage,
                                             int lane)
{
    const unsigned long long need = __ballot(ln.parked);
    const int n = __popcll(need);
    const bool mine = ln.parked;
    const int rank = (int)lanes_below(need);
    float f[9];
    if (mine) event_features(v, ln, !ln.emis_dir, f);
    for (int sb = 0; 16 * sb < n; ++sb) {
        const bool in_block = mine && (rank >> 4) == sb;
        if (in_block) {
            uint16_t *row = feat + 16 * (rank & 15);
#pragma unroll
            for (int i = 0; i < 16; ++i) row[i] = i < 9 ? bf16_bits(f[i]) : (uint16_t)0;
        }
        wave_lds_sync();
        bf16x4 x = *reinterpret_cast<const bf16x4 *>(feat + 16 * (lane & 15) + 4 * (lane >> 4));
        f32x4 o[3];
        mlp_forward16<false>(Wf, bias, x, lane, o);
#pragma unroll
        for (int t = 0; t < 3; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int row = 16 * t + 4 * (lane >> 4) + i;
                if (row < 40) stage[(lane & 15) * 41 + row] = o[t][i];
            }
        wave_lds_sync();
        if (in_block) apply_proposal<DevSink<true, false>>(v, ln, ty, stage + (rank & 15) * 41);
        wave_lds_sync();
    }
}

// LEARN: learned proposal; HIST: plain run recording histories.  A variant
// carries only the code (and registers) of its own features.
template <typename Real, typename ImgT, int G, bool LEARN, bool HIST>
__device__ __forceinline__ void transport_body(const TransportArgs<Real, ImgT, G> &a)
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
    // learned proposal (FP32): network fragments and biases in LDS, plus a
    // feature tile [16][16] bf16 and an output tile [16][41] FP32 per wave
    constexpr bool kMfma = LEARN && sizeof(Real) == 4;
    __shared__ bf16x4 s_wf[kMfma ? kFragFwd * 64 : 1];
    __shared__ float s_bias[kMfma ? kBiasFloats : 1];
    __shared__ __attribute__((aligned(16))) uint16_t s_feat[kMfma ? (kBlock / 64) * 256 : 1];
    __shared__ float s_stage[kMfma ? (kBlock / 64) * 16 * 41 : 1];
    if constexpr (kMfma) {
        const bf16x4 *wf = reinterpret_cast<const bf16x4 *>(a.mlp_frags);
        for (int i = threadIdx.x; i < kFragFwd * 64; i += blockDim.x) s_wf[i] = wf[i];
        for (int i = threadIdx.x; i < kBiasFloats; i += blockDim.x) s_bias[i] = a.mlp_bias[i];
    }
    __syncthreads();

    // Segments per march iteration: FP32 8 (4 with the learned proposal,
    // whose network needs the registers), FP64 as the host simulator.  FP32 deposits are issued transposed through LDS:
    // Cartesian runs hold their open run (16 slots per lane); octree runs and
    // the learned proposal (registers, LDS) take one slot per segment -- on
    // the octree's smaller tables the extra issue costs more than the held
    // runs save.
    //
    // A flush's atomics stay in the wave's count of outstanding vector memory
    // operations, which retire in order: the next load the wave waits for
    // (on the octree, the first walk load of the next iteration) also waits
    // until every atomic of the flush has been acknowledged by the memory
    // side.  Octree runs therefore hold no runs but take 2 kK slots, and the
    // wave flushes only when a lane could overflow in the next iteration or
    // when it leaves the march loop: every other iteration.
    constexpr int kK = sizeof(Real) != 4 ? BatchOf<G>::value
                                         : (G == kCartesian ? (LEARN ? 4 : 8) : (LEARN ? 4 : 8));
    constexpr bool kLazy = sizeof(Real) == 4 && G == kOctree;
    constexpr int kTR = sizeof(Real) == 4 ? (kLazy ? 2 * kK : (G == kCartesian && !LEARN ? 16 : kK)) : 0;
    typedef DevSink<LEARN, HIST, kTR, kK, !kLazy> SinkT;
    constexpr int kTile = kTR ? kTR * SinkT::kPitch : 1;
    __shared__ uint32_t s_tc[kTR ? (kBlock / 64) * kTile : 1];
    __shared__ float s_tv[kTR ? (kBlock / 64) * kTile : 1];
    __shared__ __attribute__((aligned(16))) uint32_t s_word[kTR ? kBlock : 4];
    const int lane = __lane_id();
    const int wave = threadIdx.x >> 6;
    SinkT sink;
    if constexpr (kTR > 0) {
        sink.sc = s_tc + wave * kTile + lane;
        sink.sv = s_tv + wave * kTile + lane;
    }
    Lane<Real> ln;
    ln.mode = kDead;
    ln.marching = false;
    ln.parked = false;
    ln.pix = -1;
    Tally ty = {};
    __shared__ PixelCarry s_carry[kBlock / 64];
    PixelCarry *carry = s_carry + wave;
    carry_init(carry, lane);
    uint64_t cur = 0, end = 0;
    bool exhausted = false;

    for (;;) {
        // refill dead lanes from the wave's chunk (one atomic per chunk); a
        // refilled lane only launches here, its events run below
        bool launched = false;
        for (;;) {
            unsigned long long dead = __ballot(ln.mode == kDead && !ln.parked && !launched);
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
            if (ln.mode == kDead && !ln.parked && !launched && (uint64_t)rank < avail) {
                uint64_t P = cur + rank;
                uint32_t lam = (uint32_t)(P / a.count);
                uint32_t id = (uint32_t)(a.first_id + P % a.count);
                launch<decltype(sink)>(v, ln, ty, lam, id, (uint32_t)P);
                launched = true;
            }
            uint64_t ndead = (uint64_t)__popcll(dead);
            cur += ndead < avail ? ndead : avail;
        }
        // events of the lanes whose march ended (or that just launched); with
        // the learned proposal, the lanes parked for a direction get it here
        for (;;) {
            if (!ln.marching && ln.mode != kDead) settle(v, ln, ty, sink);
            if constexpr (!LEARN) {
                break;
            } else {
                if (__ballot(ln.parked) == 0) break;
                if constexpr (kMfma) {
                    resolve_wave(v, ln, ty, s_wf, s_bias, s_feat + wave * 256, s_stage + wave * 16 * 41, lane);
                } else {
                    if (ln.parked) resolve_direction_scalar<decltype(sink)>(v, ln, ty);
                }
            }
        }
        flush_pixels(ln, v.images, lane, carry);
        if (__ballot(ln.mode != kDead) == 0) {
            if (exhausted) break;
            continue;
        }

        // march: every marching lane advances kK cells per iteration; the
        // iteration's deposits go out after it
        for (;;) {
            if (ln.marching) march_batch<kK>(v, ln, ty, sink);
            unsigned long long waiting = __ballot(!ln.marching && (ln.mode != kDead || !exhausted));
            unsigned long long active = __ballot(ln.marching);
            const bool leave = active == 0 || __popcll(waiting) >= a.threshold;
            // a lane's wavelength changes only after the loop: the slots may
            // wait across iterations, never across a relaunch
            if (!kLazy || leave || sink.must_flush())
                sink.flush(lane, ln.marching && ln.mode == kProp, (int)ln.lam, v.table, v.n_store,
                           s_tc + wave * kTile, s_tv + wave * kTile, s_word + wave * 64);
            if (leave) break;
        }
    }

    flush_carry(carry, v.images, lane);
    double e0 = wave_sum(ty.emitted), e1 = wave_sum(ty.absorbed);
    double e2 = wave_sum(ty.escaped), e3 = wave_sum(ty.truncated);
    unsigned long long s[kNumStats] = {ty.packets, ty.events, ty.prop_cells, ty.locate_cells,
                                       ty.peel_cells, ty.peel_adds, ty.peel_dropped, ty.capped,
                                       ty.guard, ty.nonfinite};
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

// FP32 production kernels: at most 168 VGPRs, three waves per SIMD; the
// plain octree kernel, bound by the latency of its walk's dependent loads,
// four waves per SIMD (128 VGPRs, a few registers spilled).
template <int G, bool LEARN, bool HIST>
__global__ void __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(G == kOctree && !LEARN && !HIST ? 4 : 3)))
transport_kernel_f32(TransportArgs<float, float, G> a)
{
    transport_body<float, float, G, LEARN, HIST>(a);
}

// FP64 validation kernels (the scalar FP64 network needs more registers).
template <int G, bool LEARN, bool HIST>
__global__ void __launch_bounds__(kBlock) transport_kernel_f64(TransportArgs<double, double, G> a)
{
    transport_body<double, double, G, LEARN, HIST>(a);
}

template <typename Real, typename ImgT, int G>
__device__ __forceinline__ void flush_tally(Tally &ty, double *energy, unsigned long long *stats, int lane)
{
    double e0 = wave_sum(ty.emitted), e1 = wave_sum(ty.absorbed);
    double e2 = wave_sum(ty.escaped), e3 = wave_sum(ty.truncated);
    unsigned long long s[kNumStats] = {ty.packets, ty.events, ty.prop_cells, ty.locate_cells,
                                       ty.peel_cells, ty.peel_adds, ty.peel_dropped, ty.capped,
                                       ty.guard, ty.nonfinite};
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
template <typename Real, typename ImgT, int SLOTS>
__device__ __forceinline__ void batch_body(const BatchArgs<Real, ImgT> &a,
                                           const ModelDesc<Real, ImgT> *__restrict__ models)
{
    // one deposit slot per segment (the batch's small tables stay in the L2,
    // where holding runs does not pay for its extra issue).  SLOTS (FP32) is
    // the tile per lane, a tuning choice: kK slots, issued after every march
    // iteration, or 2 kK, issued only when a lane could overflow or the wave
    // leaves the march loop (as in the octree kernels: a flush's atomics
    // delay the next loads the wave waits for)
    constexpr int kK = sizeof(Real) == 4 ? 8 : BatchOf<0>::value;
    constexpr int kTR = sizeof(Real) == 4 ? SLOTS : 0;
    static_assert(sizeof(Real) != 4 || SLOTS == kK || SLOTS == 2 * kK, "deposit tile");
    constexpr bool kLazyB = kTR == 2 * kK;
    typedef DevSink<false, false, kTR, kK, false> SinkT;
    constexpr int kTile = kTR ? kTR * SinkT::kPitch : 1;
    __shared__ uint32_t s_tc[kTR ? (kBlock / 64) * kTile : 1];
    __shared__ float s_tv[kTR ? (kBlock / 64) * kTile : 1];
    __shared__ __attribute__((aligned(16))) uint32_t s_word[kTR ? kBlock : 4];
    const int wave = threadIdx.x >> 6;
    const int lane = __lane_id();
    SinkT sink;
    if constexpr (kTR > 0) {
        sink.sc = s_tc + wave * kTile + lane;
        sink.sv = s_tv + wave * kTile + lane;
    }
    Lane<Real> ln;
    ln.mode = kDead;
    ln.marching = false;
    ln.pix = -1;
    Tally ty = {};
    __shared__ PixelCarry s_carry[kBlock / 64];
    PixelCarry *carry = s_carry + wave;
    carry_init(carry, lane);
    int cur_model = -1, pend_model = -1;
    // The current model's view is read through a constant-address-space
    // pointer formed from a wave-uniform model index at every use: its fields
    // become scalar loads the compiler may repeat instead of holding ~60
    // values in registers across the event loop (a pointer carried across
    // the queue loop is not provably uniform, and its loads go to the vector
    // memory path).
    typedef const View<Real, ImgT, 0> __attribute__((address_space(4))) CView;
    auto V = [&]() -> const View<Real, ImgT, 0> & {
        const int m = __builtin_amdgcn_readfirstlane(cur_model < 0 ? 0 : cur_model);
        return models[m].view;
    };
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
                    if (cur_model >= 0) {
                        flush_carry(carry, V().images, lane);
                        flush_tally<Real, ImgT, 0>(ty, a.models[cur_model].energy, a.models[cur_model].stats, lane);
                    }
                    cur_model = pend_model;
                    const ModelDesc<Real, ImgT> &m = a.models[cur_model];
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
                launch<decltype(sink)>(V(), ln, ty, (uint32_t)(P / count), (uint32_t)(first_id + P % count), (uint32_t)P);
                launched = true;
            }
            uint64_t ndead = (uint64_t)__popcll(dead);
            cur += ndead < avail ? ndead : avail;
        }
        if (!ln.marching && ln.mode != kDead) settle(V(), ln, ty, sink);
        flush_pixels(ln, V().images, lane, carry);
        if (__ballot(ln.mode != kDead) == 0) {
            if (exhausted) break;
            continue;
        }
        for (;;) {
            if (ln.marching) march_batch<kK>(V(), ln, ty, sink);
            unsigned long long waiting = __ballot(!ln.marching && (ln.mode != kDead || !exhausted));
            unsigned long long active = __ballot(ln.marching);
            const bool leave = active == 0 || __popcll(waiting) >= a.threshold;
            if (!kLazyB || leave || sink.must_flush())
                sink.flush(lane, ln.marching && ln.mode == kProp, (int)ln.lam, V().table, V().n_store,
                           s_tc + wave * kTile, s_tv + wave * kTile, s_word + wave * 64);
            if (leave) break;
        }
    }
    if (cur_model >= 0) {
        flush_carry(carry, V().images, lane);
        flush_tally<Real, ImgT, 0>(ty, a.models[cur_model].energy, a.models[cur_model].stats, lane);
    }
}

// FP32: four waves per SIMD (128 VGPRs, a few registers spilled): the
// event-heavy batch gains more from the extra wave than the spills cost.
template <typename ImgT, int SLOTS>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
batch_transport_kernel_f32(BatchArgs<float, ImgT> a, const ModelDesc<float, ImgT> *__restrict__ models)
{
    batch_body<float, ImgT, SLOTS>(a, models);
}

template <typename ImgT>
__global__ void __launch_bounds__(kBlock) batch_transport_kernel_f64(BatchArgs<double, ImgT> a, const ModelDesc<double, ImgT> *__restrict__ models)
{
    batch_body<double, ImgT, 0>(a, models);
}

template <typename Real, typename ImgT, int SLOTS>
hipError_t launch_batch_impl(const BatchArgs<Real, ImgT> &a, int grid, hipStream_t stream)
{
    if constexpr (sizeof(Real) == 4)
        hipLaunchKernelGGL((batch_transport_kernel_f32<ImgT, SLOTS>), dim3(grid), dim3(kBlock), 0, stream, a,
                           a.models);
    else
        hipLaunchKernelGGL(batch_transport_kernel_f64<ImgT>, dim3(grid), dim3(kBlock), 0, stream, a, a.models);
    return hipGetLastError();
}

template <typename Real, typename ImgT, int G>
hipError_t launch_transport_impl(const TransportArgs<Real, ImgT, G> &a, int grid, hipStream_t stream)
{
    if constexpr (sizeof(Real) == 4) {
        if (a.view.learned)
            hipLaunchKernelGGL((transport_kernel_f32<G, true, false>), dim3(grid), dim3(kBlock), 0, stream, a);
        else if (a.view.hist)
            hipLaunchKernelGGL((transport_kernel_f32<G, false, true>), dim3(grid), dim3(kBlock), 0, stream, a);
        else
            hipLaunchKernelGGL((transport_kernel_f32<G, false, false>), dim3(grid), dim3(kBlock), 0, stream, a);
    } else {
        if (a.view.learned)
            hipLaunchKernelGGL((transport_kernel_f64<G, true, false>), dim3(grid), dim3(kBlock), 0, stream, a);
        else if (a.view.hist)
            hipLaunchKernelGGL((transport_kernel_f64<G, false, true>), dim3(grid), dim3(kBlock), 0, stream, a);
        else
            hipLaunchKernelGGL((transport_kernel_f64<G, false, false>), dim3(grid), dim3(kBlock), 0, stream, a);
    }
    return hipGetLastError();
}

} // namespace mcrt
