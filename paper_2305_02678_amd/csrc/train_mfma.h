// Differentiation of the decode on the gfx950 matrix cores (FP32 v_mfma_f32_16x16x4_f32):
// training by backpropagation into the decoder and directly into the latent texels (Sec. 5 and
// the direct optimisation of Sec. 2 "Obtaining latent textures"), for decoders C+6 -> H -> ... -> H
// -> NO with C in {8, 16}, H in {32, 64}, 2 or 3 hidden layers, NO in {3, 6}.
//
// Work decomposition.  One workgroup of 4 waves per CU; every wave walks its own 16-sample
// tiles and does everything for a tile: fetch, forward, backward, the weight gradients and the
// latent scatter.  The decoder's operand blocks (below) sit in LDS, shared by the 4 waves; each
// wave has a private LDS scratch with its tile's activations in sample-major order.
//
// Lane (g, s) = (lane / 16, lane % 16) works on sample s of the tile.  A layer is
// Y = W X with the weights as the A operand (16 output rows per row tile) and one sample per
// column; its accumulator leaves lane (g, s) holding rows 4g..4g+3 of each row tile.  The next
// layer takes K steps (t, r) = {16t + 4g + r : g = 0..3}, so the accumulator registers [t][r]
// are exactly its B operands: the weights' K order is permuted when they are packed, and no
// activation moves between lanes.  The backward products W^T delta use the same trick with the
// packed transposes.  The weight gradients dW = delta a^T contract over the samples, which sit
// on the accumulator's columns; both operands are read back from the sample-major LDS copies
// with samples on the K index, and the gradients accumulate in registers over all tiles of
// the wave.  At the end each wave writes its gradients to its own slice of a partial buffer,
// reduced in a fixed order afterwards, so parameter gradients do not depend on scheduling.
//
// Layer 1 input.  For the fetch, lane (g, s) loads channels 4g..4g+3 of the 8 trilinear taps of
// sample s (C = 16; for C = 8 lanes g < 2 load, lanes g >= 2 carry the directions), and its
// registers become the K slots (q, g) of layer 1 directly (slot_input).  A constant-1 slot makes
// the first layer's bias part of its weights, so dW_1 yields the bias gradient as one more
// column.  The gradient of the latent code leaves lane (g, s) with the same 4 channels it
// fetched, which it scatters into the same texels (FP32 atomics, or fixed-point in the
// deterministic mode).
#pragma once

#include "latent_fetch.h"
#include "train_internal.h"

namespace nam {

typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma_f32(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Input index of layer-1 K slot (q, g): 0..C-1 latent channels, C..C+5 the directions
// (wi x, y, z, wo x, y, z), C+6 the constant 1 (bias), -1 a zero slot.
template <int C>
__host__ __device__ constexpr int slot_input(int q, int g) {
    if (C == 16) {
        if (q < 4) return 4 * g + q;
        if (q == 4) return C + g;
        return g < 2 ? C + 4 + g : (g == 2 ? C + 6 : -1);
    }
    if (g < 2) return 4 * g + q;
    if (g == 2) return C + q;
    return q < 2 ? C + 4 + q : (q == 2 ? C + 6 : -1);
}

// Operand blocks of the decoder in LDS (floats) and the per-wave scratch.  A block of 4
// consecutive K steps is 64 lanes x 4 floats, one 16-byte read per lane.
template <int C, int H, int NH>
struct TrainLayout {
    static constexpr int HT = H / 16;              // row tiles of a hidden layer
    static constexpr int Q1 = (C + 8) / 4;         // K steps of layer 1
    static constexpr int G1 = (Q1 + 3) / 4;        // groups of 4 K steps of layer 1
    static constexpr int NCT1 = (C + 8 + 15) / 16; // column tiles of dW_1 (inputs, 1, padding)
    static constexpr int NKO = 2;                  // K steps of the output layer's transpose (NO <= 8)
    static constexpr int FW1 = 0;                                  // [t'][grp][lane][4]
    static constexpr int FWH = FW1 + HT * G1 * 256;                // layers 2..NH: [t'][t][lane][4]
    static constexpr int WH_SZ = HT * HT * 256;
    static constexpr int FWO = FWH + (NH - 1) * WH_SZ;             // [t][lane][4], rows < NO
    static constexpr int BWO = FWO + HT * 256;                     // W_out^T: [t'][q][lane]
    static constexpr int BWH = BWO + HT * NKO * 64;                // W_k^T, k = 2..NH: [t'][t][lane][4]
    static constexpr int BW1 = BWH + (NH - 1) * WH_SZ;             // W_1^T, latent rows: [t][lane][4]
    static constexpr int BIAS = BW1 + HT * 256;                    // layers 2..NH, output: [t][g][4]
    static constexpr int BLOB = BIAS + NH * HT * 16;
    static constexpr int FX = NCT1 * 16 + 4;       // row strides of the sample-major scratch
    static constexpr int FA = H + 4;
    static constexpr int FD = 16 + 4;
    static constexpr int SA = 16 * FX;             // X0 first, then a_1..a_NH, then delta_out
    static constexpr int SD = SA + NH * 16 * FA;
    static constexpr int SCR = SD + 16 * FD;
    static constexpr int LDS_FLOATS = BLOB + 4 * SCR;
    static_assert(BLOB % 4 == 0 && SCR % 4 == 0, "16-byte alignment of blocks");
};

// Packed parameter offsets (W_1[H][C+6], b_1, W_k[H][H], b_k, ..., W_out[NO][H], b_out).
template <int C, int H>
__host__ __device__ constexpr int param_off(int k) {   // k = 1 .. NH (hidden), NH + 1 output
    return k == 1 ? 0 : (C + 6) * H + H + (k - 2) * (H * H + H);
}

}  // namespace nam
