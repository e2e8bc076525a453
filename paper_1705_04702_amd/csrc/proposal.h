// proposal.h -- the learned direction proposal's network on the matrix cores.
//
// The network maps the 9 features of an emission or scattering event to the
// 40 parameters of an 8-lobe von Mises-Fisher mixture: 9 -> 64 -> 64 -> 40
// with ReLU, bfloat16 weights, inputs and hidden activations, FP32 sums.
// Every layer runs transposed, Z^T = W^T X^T, on bf16 MFMA tiles with the
// samples along the tile columns: the accumulator a lane holds for one 16-row
// output tile is then exactly the B operand that the next layer needs for the
// matching 16-deep slice of its reduction, so the hidden activations never
// leave the registers.
//
// MFMA 16x16x16 operand layout (lane l of a 64-lane wave, i = 0..3):
//   A[m][k]: m = l % 16, k = 4 (l / 16) + i
//   B[k][n]: k = 4 (l / 16) + i, n = l % 16
//   C[m][n]: m = 4 (l / 16) + i, n = l % 16
//
// The 64-deep reductions (layers 2 and 3, and the backward product through
// W2) run on CDNA4's 16 x 16 x 32 bf16 MFMA, two 16-deep slices 2j, 2j + 1 per
// instruction: a lane passes the concatenation of its two 16x16x16 operands
// (eight values) as A and as B.  The instruction's reduction then runs over a
// permutation of the 32 indices (element i of lane group l / 16 is index
// 16 (2j + i / 4) + 4 (l / 16) + i % 4 in both operands), which leaves the sum
// unchanged, so the fragments and the C -> B chaining are those of the
// 16-deep form.  Layer 1 (9 features, padded to 16) stays on 16x16x16.
//
// Weights live in "fragment order": fragment F holds, for each lane, the four
// bf16 values of that lane's A operand, so one 8-byte load per lane fetches a
// tile with consecutive lanes reading consecutive addresses.
//   forward  (A = W^T)   F = t            layer 1, output tile t (K padded 9 -> 16)
//                        F = 4 + 4t + kk  layer 2, output tile t, reduction slice kk
//                        F = 20 + 4t + kk layer 3, output tile t (rows >= 40 zero)
//   backward (A = W)     F = 32 + 3t + ko W3 [hidden][output], output slice ko
//                        F = 44 + 4t + kk W2 [in][out], reduction slice kk
// Biases: float [176] = b1 (64), b2 (64), b3 (40), zero padding (8).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcrt {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8_bits __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kFragFwd = 32;                // forward fragments
constexpr int kFragAll = 60;                // forward + backward fragments
constexpr int kFragElems = 64 * 4;          // bf16 values per fragment
constexpr int kBiasFloats = 176;
// parameter offsets in the flat layout W1 [9][64], b1, W2 [64][64], b2, W3 [64][40], b3
constexpr int kOffW1 = 0, kOffB1 = 576, kOffW2 = 640, kOffB2 = 4736, kOffW3 = 4800, kOffB3 = 7360;

// float -> bfloat16 bits, nearest even (finite inputs)
__device__ __forceinline__ uint16_t bf16_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// C += A B over two 16-deep slices at once: A = (a0, a1), B = (b0, b1), where
// (a0, b0) and (a1, b1) are the operands of the two slices in the 16x16x16
// layout.  A chain of MFMAs on one accumulator keeps to one form: the
// compiler issues a 16x16x16 that takes as C the accumulator a 16x16x32 has
// just written directly behind it, with no wait, and the sum then misses
// part of the first product.
__device__ __forceinline__ f32x4 mfma32(bf16x4 a0, bf16x4 a1, bf16x4 b0, bf16x4 b1, f32x4 c)
{
    const bf16x8_bits a = __builtin_shufflevector(a0, a1, 0, 1, 2, 3, 4, 5, 6, 7);
    const bf16x8_bits b = __builtin_shufflevector(b0, b1, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

__device__ __forceinline__ bf16x4 pack_bf16(float a, float b, float c, float d)
{
    bf16x4 r;
    r[0] = (short)bf16_bits(a);
    r[1] = (short)bf16_bits(b);
    r[2] = (short)bf16_bits(c);
    r[3] = (short)bf16_bits(d);
    return r;
}

__device__ __forceinline__ bf16x4 relu_bf16(f32x4 z)
{
    return pack_bf16(z[0] > 0.0f ? z[0] : 0.0f, z[1] > 0.0f ? z[1] : 0.0f, z[2] > 0.0f ? z[2] : 0.0f,
                     z[3] > 0.0f ? z[3] : 0.0f);
}

// Value of fragment element (F, lane, i) from the FP32 master parameters.
__device__ __forceinline__ float frag_value(const float *theta, int F, int lane, int i)
{
    const int r = lane & 15, q = 4 * (lane >> 4) + i;
    if (F < 4) { // W1^T: m = hidden, k = feature
        int m = 16 * F + r, k = q;
        return k < 9 ? theta[kOffW1 + k * 64 + m] : 0.0f;
    }
    if (F < 20) { // W2^T
        int t = (F - 4) >> 2, kk = (F - 4) & 3;
        int m = 16 * t + r, k = 16 * kk + q;
        return theta[kOffW2 + k * 64 + m];
    }
    if (F < 32) { // W3^T: m = output, k = hidden
        int t = (F - 20) >> 2, kk = (F - 20) & 3;
        int m = 16 * t + r, k = 16 * kk + q;
        return m < 40 ? theta[kOffW3 + k * 40 + m] : 0.0f;
    }
    if (F < 44) { // W3: m = hidden, k = output
        int t = (F - 32) / 3, ko = (F - 32) % 3;
        int m = 16 * t + r, k = 16 * ko + q;
        return k < 40 ? theta[kOffW3 + m * 40 + k] : 0.0f;
    }
    { // W2: m = input hidden, k = output hidden
        int t = (F - 44) >> 2, kk = (F - 44) & 3;
        int m = 16 * t + r, k = 16 * kk + q;
        return theta[kOffW2 + m * 64 + k];
    }
}

__device__ __forceinline__ f32x4 bias4(const float *bias, int off, int lane)
{
    const float *b = bias + off + 4 * (lane >> 4);
    f32x4 c;
    c[0] = b[0];
    c[1] = b[1];
    c[2] = b[2];
    c[3] = b[3];
    return c;
}

// Forward pass of 16 samples (the tile columns).  x: this lane's B operand of
// the input (features 4 (l/16) .. +3 of sample l % 16, zero beyond 9).
// Out: o[t] holds outputs 16 t + 4 (l/16) + i of sample l % 16; optionally the
// hidden activations (B operands) for the backward pass.
template <bool KEEP>
__device__ __forceinline__ void mlp_forward16(const bf16x4 *Wf, const float *bias, bf16x4 x, int lane, f32x4 o[3],
                                              bf16x4 *h1_out = nullptr, bf16x4 *h2_out = nullptr)
{
    bf16x4 h1[4], h2[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) h1[t] = relu_bf16(mfma16(Wf[t * 64 + lane], x, bias4(bias, 16 * t, lane)));
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 c = bias4(bias, 64 + 16 * t, lane);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            c = mfma32(Wf[(4 + 4 * t + 2 * j) * 64 + lane], Wf[(5 + 4 * t + 2 * j) * 64 + lane], h1[2 * j],
                       h1[2 * j + 1], c);
        h2[t] = relu_bf16(c);
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        f32x4 c = bias4(bias, 128 + 16 * t, lane);
#pragma unroll
        for (int j = 0; j < 2; ++j)
            c = mfma32(Wf[(20 + 4 * t + 2 * j) * 64 + lane], Wf[(21 + 4 * t + 2 * j) * 64 + lane], h2[2 * j],
                       h2[2 * j + 1], c);
        o[t] = c;
    }
    if constexpr (KEEP) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            h1_out[t] = h1[t];
            h2_out[t] = h2[t];
        }
    }
}

// Makes this wave's LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

} // namespace mcrt
