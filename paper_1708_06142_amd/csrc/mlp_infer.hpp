// Inference of the learned Ewald surrogate on the matrix cores (internal;
// shared by the surrogate walk and the column walk that carries it).
//
// Every layer runs in the transposed form h_next = W h, with the weights as
// the A operand and the 32 pairs of a batch as the columns of B, FP16 inputs
// and FP32 accumulation (v_mfma_f32_32x32x16_f16).  In that orientation the
// 32x32 output tile of one layer sits in each lane where the next layer's B
// operand needs it, up to a fixed permutation of the contraction index that
// is applied to the packed weights instead.  Biases enter as an extra
// contraction chunk against a constant (1, 1) input, split into FP16 high and
// low parts; the input scaling is folded into the first layer and the output
// de-standardisation into the last.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace ot {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace mlpdef {
// activation z S(z): S the cubic smoothstep from 0 at z = -3 to 1 at z = 3
__device__ inline float gate_t(float z) { return fminf(fmaxf(fmaf(z, 1.0f / 6.0f, 0.5f), 0.0f), 1.0f); }
__device__ inline float act(float z) {
  const float t = gate_t(z);
  return z * (t * t * fmaf(t, -2.0f, 3.0f));
}
}  // namespace mlpdef

namespace mlpinf {

using namespace mlpdef;

__device__ inline f32x16 mma(f16x8 a, f16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

// The packed operands live in LDS (27.6 KB per workgroup); each lane reads
// its 16 bytes of an operand just before the instruction that needs it, which
// keeps them out of the registers the products and activations need.
struct Ops {
  const f16x8 *lds;  // [NPK][64]
  int lane;          // this lane's slot, hidden from the compiler per call (see forward)
  __device__ f16x8 operator[](int i) const { return lds[64 * i + lane]; }
};

// all threads of the workgroup copy the operands into lds (then a barrier)
__device__ inline Ops load_ops(const void *pk, f16x8 *lds) {
  const f16x8 *p = reinterpret_cast<const f16x8 *>(pk);
  for (int i = threadIdx.x; i < 64 * NPK; i += blockDim.x) lds[i] = p[i];
  __syncthreads();
  return Ops{lds, (int)(threadIdx.x & 63)};
}

// B operand of the first layer: u split into FP16 high and low parts, with
// the constant inputs for the bias; lane group 1 passes u_hi for the low
// parts of the weights
__device__ inline f16x8 input(float u0, float u1, float u2) {
  f16x8 b;
  const bool g1 = (threadIdx.x & 63) >= 32;
  const _Float16 h0 = (_Float16)u0, h1 = (_Float16)u1, h2 = (_Float16)u2;
  const _Float16 one = (_Float16)(g1 ? 0.0f : 1.0f), zero = (_Float16)0.0f;
  b[0] = h0;
  b[1] = h1;
  b[2] = h2;
  b[3] = one;
  b[4] = g1 ? zero : (_Float16)(u0 - (float)h0);
  b[5] = g1 ? zero : (_Float16)(u1 - (float)h1);
  b[6] = g1 ? zero : (_Float16)(u2 - (float)h2);
  b[7] = one;
  return b;
}

__device__ inline f16x8 ones() {
  f16x8 b;
  const bool g0 = (threadIdx.x & 63) < 32;
  for (int j = 0; j < 8; ++j) b[j] = (_Float16)((j < 2 && g0) ? 1.0f : 0.0f);
  return b;
}

__device__ inline void act_tile(const f32x16 &d, f16x8 &c0, f16x8 &c1) {
  for (int j = 0; j < 8; ++j) {
    c0[j] = (_Float16)act(d[j]);
    c1[j] = (_Float16)act(d[8 + j]);
  }
}

// The ten channels at the folded offsets of the 32 pairs of this wave: lane l
// passes the B operand of pair l % 32 and receives its outputs (both lane
// groups receive all ten).
__device__ inline void forward(const Ops &W0, const f16x8 &xin, const f16x8 &one, float y[NO]) {
  // An empty asm makes the lane slot opaque, so the operand reads are not
  // hoisted out of the walk's loops into registers (which would leave the
  // products in accumulation registers and cut the occupancy).
  Ops W = W0;
  asm volatile("" : "+v"(W.lane));
  const f32x16 z = {0};
  f16x8 h[4];
  {
    const f32x16 d0 = mma(W[PK_L1], xin, z);
    const f32x16 d1 = mma(W[PK_L1 + 1], xin, z);
    act_tile(d0, h[0], h[1]);
    act_tile(d1, h[2], h[3]);
  }
#pragma unroll
  for (int layer = 0; layer < 2; ++layer) {
    const int A0 = layer == 0 ? PK_L2 : PK_L3, B0 = layer == 0 ? PK_L2B : PK_L3B;
    f32x16 d0 = mma(W[B0], one, z);
    f32x16 d1 = mma(W[B0 + 1], one, z);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      d0 = mma(W[A0 + c], h[c], d0);
      d1 = mma(W[A0 + 4 + c], h[c], d1);
    }
    act_tile(d0, h[0], h[1]);
    act_tile(d1, h[2], h[3]);
  }
  f32x16 o = mma(W[PK_L4B], one, z);
#pragma unroll
  for (int c = 0; c < 4; ++c) o = mma(W[PK_L4 + c], h[c], o);
  for (int k = 0; k < NO; ++k) y[k] = o[k];
}

}  // namespace mlpinf

// The surrogate walk's Taylor groups: (group, list entry) pairs per chunk of
// entries (512 single cells with one entry, else 256) and the floats each
// pair leaves in LDS (the ten channels with signs, d0 and the far flag).
__host__ __device__ inline int taylor_pairs(int gl) { return gl == 0 ? 512 : 256; }
constexpr int TSLOT = 16;

}  // namespace ot
