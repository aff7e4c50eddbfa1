// Order of the matrix-core operands of a packed decoder, shared by the host packer and the
// MFMA decode kernel.
//
// Layers are numbered 0 (input layer, C + 6 inputs padded to K = 32) to NH (output layer, 3
// rows padded to one 16-row tile).  Layer L has row tiles j (16 output neurons each) and K
// steps s (32 inputs each); every (L, j, s) is one A-operand block of 64 lanes x 16 bytes
// (8 FP16 weights, or 8 E4M3 weights in the low 8 bytes).  Lane (g, r) = (lane / 16,
// lane % 16) of a block holds row 16 j + r and K slots 8 g .. 8 g + 7 of step s.  The K slot
// (s, g, e) of layer 0 is network input 8 g + e; of a later layer it is neuron
// 16 (2 s + e / 4) + 4 g + e % 4 of the previous layer (the accumulator layout of the
// previous layer's row tiles 2 s and 2 s + 1).  Bias blocks are 64 lanes x 4 floats: lane
// (g, r) holds the biases of neurons 16 j + 4 g + 0..3, the rows of its accumulator.
#pragma once

namespace nam {

struct MfmaLayout {
    int RT, KS, NH;

    __host__ __device__ int a_blocks() const { return RT + (NH - 1) * RT * KS + KS; }
    __host__ __device__ int b_blocks() const { return NH * RT + 1; }

    __host__ __device__ int a_index(int layer, int j, int s) const {
        if (layer == 0) return j;
        if (layer < NH) return RT + (layer - 1) * RT * KS + j * KS + s;
        return RT + (NH - 1) * RT * KS + s;
    }
    __host__ __device__ int b_index(int layer, int j) const { return layer < NH ? layer * RT + j : NH * RT; }

    // neuron of the previous layer (or network input for layer 0) behind K slot (s, g, e)
    __host__ __device__ static int k_source(int layer, int s, int g, int e) {
        return layer == 0 ? 8 * g + e : 16 * (2 * s + e / 4) + 4 * g + (e % 4);
    }
};

__host__ __device__ inline MfmaLayout mfma_layout(int /*C*/, int H, int NH, bool /*l1f16*/, bool /*hf8*/) {
    return MfmaLayout{H / 16, (H + 31) / 32, NH};
}

}  // namespace nam
