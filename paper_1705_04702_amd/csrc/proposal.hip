// proposal.hip -- kernels of the learned direction proposal: parameter
// packing, batched network evaluation, the weighted-likelihood gradient
// (forward and backward on the matrix cores), the Adam step, and the
// compaction of recorded histories into training samples.
//
// Training objective: the negative log-likelihood of the vMF mixture at the
// directions a plain run actually took, each event weighted by the image flux
// its packet produced afterwards per unit of its luminosity after the event,
// normalised by the sum of those weights.
#include <hip/hip_runtime.h>

#define MCRT_HD __device__ __forceinline__
#include "transport_core.h"
#include "internal.h"
#include "proposal.h"

namespace mcrt {

// ---------------------------------------------------------------------------
// Parameters: FP32 master -> fragments (bf16), biases (FP32) and the FP64
// copy the scalar network of the FP64 validation kernel reads.
// ---------------------------------------------------------------------------
__global__ void pack_kernel(const float *theta, uint16_t *frags, float *bias, double *theta64)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kFragAll * kFragElems) {
        int F = i / kFragElems, r = i % kFragElems, lane = r >> 2, e = r & 3;
        frags[i] = bf16_bits(frag_value(theta, F, lane, e));
    }
    if (i < kBiasFloats) {
        float b = 0.0f;
        if (i < 64) b = theta[kOffB1 + i];
        else if (i < 128) b = theta[kOffB2 + i - 64];
        else if (i < 168) b = theta[kOffB3 + i - 128];
        bias[i] = b;
    }
    if (i < kMlpParams) {
        bool weight = i < kOffB1 || (i >= kOffW2 && i < kOffB2) || (i >= kOffW3 && i < kOffB3);
        theta64[i] = weight ? (double)bf16_float(bf16_bits(theta[i])) : (double)theta[i];
    }
}

hipError_t launch_proposal_pack(const float *theta, uint16_t *frags, float *bias, double *theta64,
                                hipStream_t stream)
{
    const int n = kFragAll * kFragElems; // the largest of the three ranges
    hipLaunchKernelGGL(pack_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, theta, frags, bias, theta64);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched forward pass: out[s][0..39] for features X[s][0..8].  One wave per
// 16 samples at a time; the same tile routine as inside the transport kernel.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) forward_kernel(const uint16_t *frags, const float *bias_g, const float *X,
                                                      int64_t n, float *out)
{
    __shared__ bf16x4 s_wf[kFragFwd * 64];
    __shared__ float s_bias[kBiasFloats];
    const bf16x4 *wf = reinterpret_cast<const bf16x4 *>(frags);
    for (int i = threadIdx.x; i < kFragFwd * 64; i += blockDim.x) s_wf[i] = wf[i];
    for (int i = threadIdx.x; i < kBiasFloats; i += blockDim.x) s_bias[i] = bias_g[i];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t nblk = (n + 15) / 16;
    for (int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < nblk; b += waves) {
        const int64_t s = 16 * b + (lane & 15);
        float xv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int q = 4 * (lane >> 4) + i;
            xv[i] = (s < n && q < 9) ? X[s * 9 + q] : 0.0f;
        }
        f32x4 o[3];
        mlp_forward16<false>(s_wf, s_bias, pack_bf16(xv[0], xv[1], xv[2], xv[3]), lane, o);
        if (s < n) {
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int row = 16 * t + 4 * (lane >> 4) + i;
                    if (row < 40) out[s * 40 + row] = o[t][i];
                }
        }
    }
}

hipError_t launch_proposal_forward(const uint16_t *frags, const float *bias, const float *X, int64_t n, float *out,
                                   hipStream_t stream)
{
    int64_t blocks = (n + 63) / 64;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(forward_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, frags, bias, X, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Loss gradient of one sample with respect to the 40 network outputs.
// Returns w * (-log q_vMF(kp)).  dO = d(w * -log q)/d o.
// ---------------------------------------------------------------------------
__device__ float nll_grad(const float *o, const float kp[3], float w, float *dO)
{
    const float two_pi = 6.28318530717958647692f;
    float mx = o[0];
#pragma unroll
    for (int j = 1; j < 8; ++j) mx = fmaxf(mx, o[j]);
    float e[8], sum = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        e[j] = expf(o[j] - mx);
        sum += e[j];
    }
    float pi[8], f[8], kap[8], dkds[8], dot[8], mu[8][3], nrm[8];
    float q = 0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        pi[j] = e[j] / sum;
        float a = o[8 + 3 * j], b = o[9 + 3 * j], c = o[10 + 3 * j];
        nrm[j] = sqrtf(a * a + b * b + c * c);
        if (nrm[j] > 0.0f) {
            mu[j][0] = a / nrm[j];
            mu[j][1] = b / nrm[j];
            mu[j][2] = c / nrm[j];
        } else {
            mu[j][0] = 0.0f;
            mu[j][1] = 0.0f;
            mu[j][2] = 1.0f;
        }
        float s = o[32 + j];
        float sp = log1pf(expf(-fabsf(s))) + fmaxf(s, 0.0f) + 1e-3f;
        kap[j] = fminf(fmaxf(sp, 1e-3f), 1e3f);
        dkds[j] = (sp > 1e-3f && sp < 1e3f) ? 1.0f / (1.0f + expf(-s)) : 0.0f;
        dot[j] = mu[j][0] * kp[0] + mu[j][1] * kp[1] + mu[j][2] * kp[2];
        f[j] = kap[j] / (two_pi * -expm1f(-2.0f * kap[j])) * expf(kap[j] * (dot[j] - 1.0f));
        q += pi[j] * f[j];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float r = pi[j] * f[j] / q;
        dO[j] = -w * (r - pi[j]);
        float gm = nrm[j] > 0.0f ? r * kap[j] / nrm[j] : 0.0f;
#pragma unroll
        for (int a = 0; a < 3; ++a) dO[8 + 3 * j + a] = -w * gm * (kp[a] - dot[j] * mu[j][a]);
        float e2 = expf(-2.0f * kap[j]);
        float dlogf = 1.0f / kap[j] - 2.0f * e2 / (-expm1f(-2.0f * kap[j])) + (dot[j] - 1.0f);
        dO[32 + j] = -w * r * dlogf * dkds[j];
    }
    return -w * logf(q);
}

// ---------------------------------------------------------------------------
// Gradient kernel: one wave per workgroup; each wave takes groups of 64
// samples.  Forward (4 tiles of 16 samples) keeps X^T, H1^T, H2^T (bf16) in
// LDS; each lane then forms dO for its sample; the backward pass runs on the
// matrix cores with dO and the pre-activation gradients split into bf16
// high + low parts (about 16 significant bits).  Weight gradients accumulate
// in registers across all of the wave's samples and are written once per
// wave to partial[wave][7400] (summed in a fixed order by the Adam kernel).
// ---------------------------------------------------------------------------
constexpr int kSX = 68;  // row stride (bf16) of [16 or 64 rows][64 samples] tiles
constexpr int kSO = 52;  // row stride of dO [64 samples][48 outputs]
constexpr int kSZ = 20;  // row stride of dZ [64 hidden][16 samples]
constexpr int kGradStride = kGradStrideFloats;

// Sample of position si in this pass.
__device__ __forceinline__ int64_t sample_index(const GradArgs &g, int64_t si)
{
    if (!g.random) return si;
    U4 r = philox((uint32_t)si, (uint32_t)((uint64_t)si >> 32), g.step, 0x5A4D504Cu, g.key0, g.key1);
    uint64_t w = ((uint64_t)r.x << 32) | (uint64_t)r.y;
    return (int64_t)__umul64hi(w, (uint64_t)g.n); // floor(w n / 2^64)
}

__device__ __forceinline__ bf16x4 lds4(const uint16_t *p) { return *reinterpret_cast<const bf16x4 *>(p); }

__device__ __forceinline__ void split_bf16(f32x4 x, bf16x4 &hi, bf16x4 &lo)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint16_t h = bf16_bits(x[i]);
        hi[i] = (short)h;
        lo[i] = (short)bf16_bits(x[i] - bf16_float(h));
    }
}

__global__ void __launch_bounds__(64) grad_kernel(GradArgs g)
{
    __shared__ __attribute__((aligned(16))) bf16x4 s_wf[kFragAll * 64];
    __shared__ float s_bias[kBiasFloats];
    // bf16 tiles are read 4 values (8 bytes) at a time: 16-byte aligned
    __shared__ __attribute__((aligned(16))) uint16_t s_xt[16 * kSX];
    __shared__ __attribute__((aligned(16))) uint16_t s_h1t[64 * kSX];
    __shared__ __attribute__((aligned(16))) uint16_t s_h2t[64 * kSX];
    __shared__ float s_stage[64 * 41];
    __shared__ __attribute__((aligned(16))) uint16_t s_dos_hi[64 * kSO];
    __shared__ __attribute__((aligned(16))) uint16_t s_dos_lo[64 * kSO];
    __shared__ __attribute__((aligned(16))) uint16_t s_doo_hi[48 * kSX];
    __shared__ __attribute__((aligned(16))) uint16_t s_doo_lo[48 * kSX];
    __shared__ __attribute__((aligned(16))) uint16_t s_dz2_hi[64 * kSZ];
    __shared__ __attribute__((aligned(16))) uint16_t s_dz2_lo[64 * kSZ];
    __shared__ __attribute__((aligned(16))) uint16_t s_dz1_hi[64 * kSZ];
    __shared__ __attribute__((aligned(16))) uint16_t s_dz1_lo[64 * kSZ];

    const int lane = threadIdx.x;
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(g.frags);
        uint4 *dst = reinterpret_cast<uint4 *>(s_wf);
        for (int i = lane; i < kFragAll * 32; i += 64) dst[i] = src[i];
    }
    for (int i = lane; i < kBiasFloats; i += 64) s_bias[i] = g.bias[i];
    __syncthreads();

    const int r16 = lane & 15, q4 = 4 * (lane >> 4);
    f32x4 acc3[4][3], acc2[4][4], acc1[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        acc1[a] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int b = 0; b < 3; ++b) acc3[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int b = 0; b < 4; ++b) acc2[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    float db1 = 0.0f, db2 = 0.0f, db3 = 0.0f, loss = 0.0f;

    for (int64_t grp = blockIdx.x; 64 * grp < g.m; grp += gridDim.x) {
        // ---- forward, 4 tiles of 16 samples ----
#pragma unroll 1
        for (int sb = 0; sb < 4; ++sb) {
            const int64_t si = 64 * grp + 16 * sb + r16;
            const bool valid = si < g.m;
            const int64_t id = valid ? sample_index(g, si) : 0;
            float xv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int q = q4 + i;
                xv[i] = (valid && q < 9) ? g.X[id * 9 + q] : 0.0f;
            }
            bf16x4 x = pack_bf16(xv[0], xv[1], xv[2], xv[3]);
#pragma unroll
            for (int i = 0; i < 4; ++i) s_xt[(q4 + i) * kSX + 16 * sb + r16] = (uint16_t)x[i];
            f32x4 o[3];
            bf16x4 h1[4], h2[4];
            mlp_forward16<true>(s_wf, s_bias, x, lane, o, h1, h2);
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    s_h1t[(16 * t + q4 + i) * kSX + 16 * sb + r16] = (uint16_t)h1[t][i];
                    s_h2t[(16 * t + q4 + i) * kSX + 16 * sb + r16] = (uint16_t)h2[t][i];
                }
#pragma unroll
            for (int t = 0; t < 3; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int row = 16 * t + q4 + i;
                    if (row < 40) s_stage[(16 * sb + r16) * 41 + row] = o[t][i];
                }
        }
        __syncthreads();
        // ---- per-sample loss gradient (lane = sample) ----
        {
            const int64_t si = 64 * grp + lane;
            float dO[40];
            if (si < g.m) {
                const int64_t id = sample_index(g, si);
                float kp[3] = {g.KP[id * 3 + 0], g.KP[id * 3 + 1], g.KP[id * 3 + 2]};
                float w = g.C[id] * g.scale;
                loss += nll_grad(s_stage + lane * 41, kp, w, dO);
            } else {
#pragma unroll
                for (int j = 0; j < 40; ++j) dO[j] = 0.0f;
            }
#pragma unroll
            for (int j = 0; j < 48; ++j) {
                float d = j < 40 ? dO[j] : 0.0f;
                uint16_t h = bf16_bits(d), l = bf16_bits(d - bf16_float(h));
                s_dos_hi[lane * kSO + j] = h;
                s_dos_lo[lane * kSO + j] = l;
                s_doo_hi[j * kSX + lane] = h;
                s_doo_lo[j * kSX + lane] = l;
                if (j < 40) s_stage[lane * 41 + j] = d;
            }
        }
        __syncthreads();
        if (lane < 40) {
            float sacc = 0.0f;
            for (int s = 0; s < 64; ++s) sacc += s_stage[s * 41 + lane];
            db3 += sacc;
        }
        // ---- backward, per tile of 16 samples ----
#pragma unroll 1
        for (int sb = 0; sb < 4; ++sb) {
            const int c0 = 16 * sb + q4; // sample column of this lane's k-slice
            // dW3 += H2^T dO
#pragma unroll
            for (int th = 0; th < 4; ++th) {
                bf16x4 A = lds4(s_h2t + (16 * th + r16) * kSX + c0);
#pragma unroll
                for (int to = 0; to < 3; ++to) {
                    acc3[th][to] = mfma16(A, lds4(s_doo_hi + (16 * to + r16) * kSX + c0), acc3[th][to]);
                    acc3[th][to] = mfma16(A, lds4(s_doo_lo + (16 * to + r16) * kSX + c0), acc3[th][to]);
                }
            }
            // dH2^T = W3 dO^T, masked by ReLU -> dZ2
            bf16x4 z2hi[4], z2lo[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                f32x4 c = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
                {
                    // output slices 0 and 1, high then low parts, on two 32-deep MFMAs; slice 2 (outputs
                    // 32..47) on a third that pairs the slice with itself: A = (A2, A2), B = (high, low)
                    // sums A2 high + A2 low.  One MFMA form per accumulator chain (see mfma32).
                    const bf16x4 A0 = s_wf[(32 + 3 * t) * 64 + lane], A1 = s_wf[(33 + 3 * t) * 64 + lane];
                    const bf16x4 A2 = s_wf[(34 + 3 * t) * 64 + lane];
                    const uint16_t *hi = s_dos_hi + (16 * sb + r16) * kSO + q4;
                    const uint16_t *lo = s_dos_lo + (16 * sb + r16) * kSO + q4;
                    c = mfma32(A0, A1, lds4(hi), lds4(hi + 16), c);
                    c = mfma32(A0, A1, lds4(lo), lds4(lo + 16), c);
                    c = mfma32(A2, A2, lds4(hi + 32), lds4(lo + 32), c);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (!(bf16_float(s_h2t[(16 * t + q4 + i) * kSX + 16 * sb + r16]) > 0.0f)) c[i] = 0.0f;
                split_bf16(c, z2hi[t], z2lo[t]);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    s_dz2_hi[(16 * t + q4 + i) * kSZ + r16] = (uint16_t)z2hi[t][i];
                    s_dz2_lo[(16 * t + q4 + i) * kSZ + r16] = (uint16_t)z2lo[t][i];
                }
            }
            // dH1^T = W2 dZ2^T, masked -> dZ1
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                f32x4 c = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const bf16x4 A0 = s_wf[(44 + 4 * t + 2 * j) * 64 + lane];
                    const bf16x4 A1 = s_wf[(45 + 4 * t + 2 * j) * 64 + lane];
                    c = mfma32(A0, A1, z2hi[2 * j], z2hi[2 * j + 1], c);
                    c = mfma32(A0, A1, z2lo[2 * j], z2lo[2 * j + 1], c);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (!(bf16_float(s_h1t[(16 * t + q4 + i) * kSX + 16 * sb + r16]) > 0.0f)) c[i] = 0.0f;
                bf16x4 hi, lo;
                split_bf16(c, hi, lo);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    s_dz1_hi[(16 * t + q4 + i) * kSZ + r16] = (uint16_t)hi[i];
                    s_dz1_lo[(16 * t + q4 + i) * kSZ + r16] = (uint16_t)lo[i];
                }
            }
            __syncthreads();
            // dW2 += H1^T dZ2, dW1 += X^T dZ1, bias sums
#pragma unroll
            for (int th = 0; th < 4; ++th) {
                bf16x4 A = lds4(s_h1t + (16 * th + r16) * kSX + c0);
#pragma unroll
                for (int t2 = 0; t2 < 4; ++t2) {
                    acc2[th][t2] = mfma16(A, lds4(s_dz2_hi + (16 * t2 + r16) * kSZ + q4), acc2[th][t2]);
                    acc2[th][t2] = mfma16(A, lds4(s_dz2_lo + (16 * t2 + r16) * kSZ + q4), acc2[th][t2]);
                }
            }
            {
                bf16x4 A = lds4(s_xt + r16 * kSX + c0);
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    acc1[t] = mfma16(A, lds4(s_dz1_hi + (16 * t + r16) * kSZ + q4), acc1[t]);
                    acc1[t] = mfma16(A, lds4(s_dz1_lo + (16 * t + r16) * kSZ + q4), acc1[t]);
                }
            }
            {
                float a2 = 0.0f, a1 = 0.0f;
                for (int s = 0; s < 16; ++s) {
                    a2 += bf16_float(s_dz2_hi[lane * kSZ + s]) + bf16_float(s_dz2_lo[lane * kSZ + s]);
                    a1 += bf16_float(s_dz1_hi[lane * kSZ + s]) + bf16_float(s_dz1_lo[lane * kSZ + s]);
                }
                db2 += a2;
                db1 += a1;
            }
            __syncthreads();
        }
    }

    // ---- this wave's gradient ----
    float *p = g.partial + (int64_t)blockIdx.x * kGradStride;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int f = q4 + i, h = 16 * t + r16;
            if (f < 9) p[kOffW1 + f * 64 + h] = acc1[t][i];
        }
#pragma unroll
    for (int th = 0; th < 4; ++th)
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2)
#pragma unroll
            for (int i = 0; i < 4; ++i) p[kOffW2 + (16 * th + q4 + i) * 64 + 16 * t2 + r16] = acc2[th][t2][i];
#pragma unroll
    for (int th = 0; th < 4; ++th)
#pragma unroll
        for (int to = 0; to < 3; ++to)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int o = 16 * to + r16;
                if (o < 40) p[kOffW3 + (16 * th + q4 + i) * 40 + o] = acc3[th][to][i];
            }
    p[kOffB1 + lane] = db1;
    p[kOffB2 + lane] = db2;
    if (lane < 40) p[kOffB3 + lane] = db3;
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
    if (lane == 0) g.loss_partial[blockIdx.x] = (double)loss;
}

hipError_t launch_proposal_grad(const GradArgs &g, int waves, hipStream_t stream)
{
    hipLaunchKernelGGL(grad_kernel, dim3(waves), dim3(64), 0, stream, g);
    return hipGetLastError();
}

// Sum of the per-wave gradients in a fixed order (32 parameters x 8 wave
// slices per workgroup, slices combined in index order), then optionally one
// Adam step on the FP32 master parameters.  step >= 1 is the Adam time step.
__global__ void __launch_bounds__(256) adam_kernel(const float *partial, int waves, const double *loss_partial,
                                                   AdamArgs a)
{
    __shared__ float red[8][32];
    const int c = threadIdx.x & 31, j = threadIdx.x >> 5;
    const int i = blockIdx.x * 32 + c;
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.loss_out) {
        double l = 0.0;
        for (int w = 0; w < waves; ++w) l += loss_partial[w];
        *a.loss_out = l;
    }
    float s = 0.0f;
    if (i < kMlpParams)
        for (int w = j; w < waves; w += 8) s += partial[(int64_t)w * kGradStride + i];
    red[j][c] = s;
    __syncthreads();
    if (j != 0 || i >= kMlpParams) return;
    float gsum = red[0][c];
#pragma unroll
    for (int k = 1; k < 8; ++k) gsum += red[k][c];
    if (a.grad_out) a.grad_out[i] = gsum;
    if (!a.update) return;
    float m = a.b1 * a.m[i] + (1.0f - a.b1) * gsum;
    float v = a.b2 * a.v[i] + (1.0f - a.b2) * gsum * gsum;
    a.m[i] = m;
    a.v[i] = v;
    float mh = m / (1.0f - powf(a.b1, (float)a.step));
    float vh = v / (1.0f - powf(a.b2, (float)a.step));
    a.theta[i] -= a.lr * mh / (sqrtf(vh) + a.eps);
}

hipError_t launch_proposal_adam(const float *partial, int waves, const double *loss_partial, const AdamArgs &a,
                                hipStream_t stream)
{
    hipLaunchKernelGGL(adam_kernel, dim3((kMlpParams + 31) / 32), dim3(256), 0, stream, partial, waves,
                       loss_partial, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Histories -> training samples.  Record (slot, e) is an event when its
// luminosity is positive; its weight is C = (packet total - flux so far) / L.
// Samples with C > 0 are kept, in (slot, event) order: a count per slot, an
// exclusive scan over slots, then the writes.
// ---------------------------------------------------------------------------
template <typename Real>
__device__ __forceinline__ float hist_weight(const Real *h, const Real *tot, int64_t slot, int E, int e)
{
    const Real *r = h + (slot * E + e) * kHistFloats;
    if (!(r[12] > Real(0))) return 0.0f;
    return (float)((tot[slot] - r[13]) / r[12]);
}

template <typename Real>
__global__ void hist_count_kernel(const Real *h, const Real *tot, int64_t n_slots, int E, uint32_t *count)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slots) return;
    uint32_t c = 0;
    for (int e = 0; e < E; ++e) c += hist_weight(h, tot, s, E, e) > 0.0f ? 1u : 0u;
    count[s] = c;
}

// Exclusive scan in three passes over blocks of 1024 elements.
__global__ void scan_block_kernel(const uint32_t *in, uint64_t *out, int64_t n, uint64_t *block_sums)
{
    __shared__ uint64_t s[1024];
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    uint64_t v = i < n ? in[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        uint64_t t = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = s[threadIdx.x] - v;
    if (threadIdx.x == 1023) block_sums[blockIdx.x] = s[1023];
}

__global__ void scan_sums_kernel(uint64_t *block_sums, int64_t nb, uint64_t *total)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t run = 0;
    for (int64_t b = 0; b < nb; ++b) {
        uint64_t v = block_sums[b];
        block_sums[b] = run;
        run += v;
    }
    *total = run;
}

__global__ void scan_add_kernel(uint64_t *out, int64_t n, const uint64_t *block_sums)
{
    const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (i < n) out[i] += block_sums[blockIdx.x];
}

template <typename Real>
__global__ void hist_write_kernel(const Real *h, const Real *tot, int64_t n_slots, int E, const uint64_t *offset,
                                  float *X, float *KP, float *C)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_slots) return;
    uint64_t k = offset[s];
    for (int e = 0; e < E; ++e) {
        float c = hist_weight(h, tot, s, E, e);
        if (!(c > 0.0f)) continue;
        const Real *r = h + (s * E + e) * kHistFloats;
        for (int j = 0; j < 9; ++j) X[k * 9 + j] = (float)r[j];
        for (int j = 0; j < 3; ++j) KP[k * 3 + j] = (float)r[9 + j];
        C[k] = c;
        ++k;
    }
}

template <typename Real>
hipError_t hist_count_impl(const Real *h, const Real *tot, int64_t n_slots, int E, uint32_t *count, uint64_t *offset,
                           uint64_t *block_sums, uint64_t *total, hipStream_t st)
{
    const unsigned nb = (unsigned)((n_slots + 1023) / 1024);
    hipLaunchKernelGGL((hist_count_kernel<Real>), dim3((unsigned)((n_slots + 255) / 256)), dim3(256), 0, st, h, tot,
                       n_slots, E, count);
    hipLaunchKernelGGL(scan_block_kernel, dim3(nb), dim3(1024), 0, st, count, offset, n_slots, block_sums);
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(64), 0, st, block_sums, (int64_t)nb, total);
    hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(1024), 0, st, offset, n_slots, block_sums);
    return hipGetLastError();
}

template <typename Real>
hipError_t hist_write_impl(const Real *h, const Real *tot, int64_t n_slots, int E, const uint64_t *offset, float *X,
                           float *KP, float *C, hipStream_t st)
{
    hipLaunchKernelGGL((hist_write_kernel<Real>), dim3((unsigned)((n_slots + 255) / 256)), dim3(256), 0, st, h, tot,
                       n_slots, E, offset, X, KP, C);
    return hipGetLastError();
}

hipError_t launch_hist_count(const void *h, const void *tot, bool fp64, int64_t n_slots, int E, uint32_t *count,
                             uint64_t *offset, uint64_t *block_sums, uint64_t *total, hipStream_t st)
{
    if (fp64)
        return hist_count_impl((const double *)h, (const double *)tot, n_slots, E, count, offset, block_sums, total, st);
    return hist_count_impl((const float *)h, (const float *)tot, n_slots, E, count, offset, block_sums, total, st);
}

hipError_t launch_hist_write(const void *h, const void *tot, bool fp64, int64_t n_slots, int E,
                             const uint64_t *offset, float *X, float *KP, float *C, hipStream_t st)
{
    if (fp64) return hist_write_impl((const double *)h, (const double *)tot, n_slots, E, offset, X, KP, C, st);
    return hist_write_impl((const float *)h, (const float *)tot, n_slots, E, offset, X, KP, C, st);
}

// Sum of n floats in FP64 by one workgroup, in a fixed order.
__global__ void sum_f32_kernel(const float *x, int64_t n, double *out)
{
    __shared__ double s[1024];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) a += (double)x[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

hipError_t launch_sum_f32(const float *x, int64_t n, double *out, hipStream_t stream)
{
    hipLaunchKernelGGL(sum_f32_kernel, dim3(1), dim3(1024), 0, stream, x, n, out);
    return hipGetLastError();
}

} // namespace mcrt
