// Learned surrogate of the Ewald correction.  It is not part of the paper: it
// stands in for the look-up table of Sec. 2.2.5, which stays the fallback and
// the judge of its error.
//
// Network 3 -> 64 -> 64 -> 64 -> 10 with the activation f(z) = z S(z), S the
// cubic smoothstep from 0 at z = -3 to 1 at z = 3, after each hidden layer.
// Input: the folded offset u (all components >= 0) scaled to [-1, 1] per
// axis; output: the table's ten channels (phi_c, A_c and the six second
// derivatives of phi_c) standardised per channel.  Parameters (9226 FP32):
//   W1[64][3] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[10][64] b4[10].
//
// Training (FP32): one workgroup runs forward and backward for 8 samples with
// all activations in LDS and writes its partial gradient; a second kernel sums
// the partials in a fixed order (deterministic) and applies Adam.
// Loss: mean squared error over the 10 outputs of the batch.
//
// Inference: every layer runs on the matrix cores in the transposed form
// h_next = W h, with the weights as the A operand and the 32 pairs of a batch
// as the columns of B, FP16 inputs and FP32 accumulation
// (v_mfma_f32_32x32x16_f16).  In that orientation the 32x32 output tile of one
// layer sits in each lane where the next layer's B operand needs it, up to a
// fixed permutation of the contraction index that is applied to the packed
// weights instead.  Biases enter as an extra contraction chunk against a
// constant (1, 1) input, split into FP16 high and low parts; the input scaling
// is folded into the first layer and the output de-standardisation into the
// last.  In the first layer the offset and the weights are both split into
// FP16 high and low parts (the three products that matter fill the 16-deep
// contraction), so the inputs lose no precision to FP16; the hidden
// activations and the other weights are rounded to FP16.
#include <mutex>

#include "common.hpp"
#include "ewald_lookup.hpp"
#include "kernels.hpp"
#include "mlp_infer.hpp"

namespace ot {

namespace {

using namespace mlpdef;


__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// counter-based uniform in [0, 1): stream `seed`, counter i
__device__ inline double uniform01(uint64_t seed, uint64_t i) {
  return (double)(splitmix64(splitmix64(seed) + i) >> 11) * 0x1.0p-53;
}

// f'(z) = S(z) + z t (1 - t)
__device__ inline float dact(float z) {
  const float t = gate_t(z);
  return t * t * fmaf(t, -2.0f, 3.0f) + z * t * (1.0f - t);
}

// He-uniform weights, zero biases
__global__ void k_mlp_init(uint64_t seed, float *__restrict__ P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NP) return;
  float a = 0.0f;
  if (i < OB1) a = sqrtf(6.0f / NI);
  else if ((i >= OW2 && i < OB2) || (i >= OW3 && i < OB3) || (i >= OW4 && i < OB4)) a = sqrtf(6.0f / H);
  P[i] = a == 0.0f ? 0.0f : (float)((2.0 * uniform01(seed, i) - 1.0) * a);
}

// sample offsets uniform in the folded domain [0, ext]^3
__global__ void k_mlp_points(uint64_t seed, int64_t n, double e0, double e1, double e2, double *__restrict__ u) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  u[3 * q] = e0 * uniform01(seed, 3 * q);
  u[3 * q + 1] = e1 * uniform01(seed, 3 * q + 1);
  u[3 * q + 2] = e2 * uniform01(seed, 3 * q + 2);
}

// network inputs x = 2 u / ext - 1 and the ten standardised targets
__global__ void k_mlp_prepare(int64_t n, const double *__restrict__ u, const double *__restrict__ ser,
                              MlpNorm N, float *__restrict__ x, float *__restrict__ t) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  for (int k = 0; k < 3; ++k) x[3 * q + k] = (float)(2.0 * u[3 * q + k] / N.ext[k] - 1.0);
  for (int o = 0; o < NO; ++o) t[NO * q + o] = (float)((ser[10 * q + o] - N.mu[o]) / N.sig[o]);
}

// ------------------------------------------------------------- training
constexpr int SB = 8;   // samples per workgroup (batch 2048 -> 256 workgroups)
constexpr int WP = 65;  // padded LDS row stride of W2, W3

struct TrainLds {
  float w2[H * WP], w3[H * WP];
  float z1[SB][H], z2[SB][H], z3[SB][H];
  float h1[SB][H], h2[SB][H], h3[SB][H];
  float da[SB][H], db[SB][H];
  float x[SB][NI], dy[SB][NO];
  float loss[256];
};

// Thread t: neuron o = t % 64 of samples s = t / 64 + 4 j in the layer loops.
__global__ __launch_bounds__(256) void k_mlp_fwdbwd(const float *__restrict__ P, int64_t n, int64_t s0,
                                                    const float *__restrict__ X, const float *__restrict__ T,
                                                    float scale, float *__restrict__ partial,
                                                    float *__restrict__ lossp) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TrainLds &L = *reinterpret_cast<TrainLds *>(smem_raw);
  const int t = threadIdx.x;
  const int64_t base = (s0 + (int64_t)blockIdx.x * SB) % n;  // n and s0 are multiples of SB
  for (int q = t; q < H * H; q += 256) {
    L.w2[(q / H) * WP + q % H] = P[OW2 + q];
    L.w3[(q / H) * WP + q % H] = P[OW3 + q];
  }
  for (int q = t; q < SB * NI; q += 256) L.x[q / NI][q % NI] = X[NI * base + q];
  __syncthreads();
  const int o = t % H, s4 = t / H;
  for (int j = 0; j < SB / 4; ++j) {
    const int s = s4 + 4 * j;
    float a = P[OB1 + o];
    for (int i = 0; i < NI; ++i) a += P[OW1 + o * NI + i] * L.x[s][i];
    L.z1[s][o] = a;
    L.h1[s][o] = act(a);
  }
  __syncthreads();
  // two samples per thread, s4 and s4 + 4, sharing each weight read (each
  // sum in the same order as one sample at a time)
  static_assert(SB == 8, "two samples per thread below");
  {
    const int s = s4, u = s4 + 4;
    float a = P[OB2 + o], c = a;
    for (int i = 0; i < H; ++i) {
      const float wv = L.w2[o * WP + i];
      a += wv * L.h1[s][i];
      c += wv * L.h1[u][i];
    }
    L.z2[s][o] = a;
    L.h2[s][o] = act(a);
    L.z2[u][o] = c;
    L.h2[u][o] = act(c);
  }
  __syncthreads();
  {
    const int s = s4, u = s4 + 4;
    float a = P[OB3 + o], c = a;
    for (int i = 0; i < H; ++i) {
      const float wv = L.w3[o * WP + i];
      a += wv * L.h2[s][i];
      c += wv * L.h2[u][i];
    }
    L.z3[s][o] = a;
    L.h3[s][o] = act(a);
    L.z3[u][o] = c;
    L.h3[u][o] = act(c);
  }
  __syncthreads();
  float lsum = 0.0f;
  if (t < SB * NO) {
    const int s = t / NO, oo = t % NO;
    float a = P[OB4 + oo];
    for (int i = 0; i < H; ++i) a += P[OW4 + oo * H + i] * L.h3[s][i];
    const float e = a - T[NO * (base + s) + oo];
    lsum = e * e * scale;
    L.dy[s][oo] = 2.0f * e * scale;
  }
  L.loss[t] = lsum;
  __syncthreads();
  float *G = partial + (int64_t)blockIdx.x * NP;
  {  // layer 4: dW4, db4
    for (int q = t; q < NO * H; q += 256) {
      const int oo = q / H, i = q % H;
      float g = 0.0f;
      for (int s = 0; s < SB; ++s) g += L.dy[s][oo] * L.h3[s][i];
      G[OW4 + oo * H + i] = g;
    }
    if (t < NO) {
      float gb = 0.0f;
      for (int s = 0; s < SB; ++s) gb += L.dy[s][t];
      G[OB4 + t] = gb;
    }
  }
  for (int j = 0; j < SB / 4; ++j) {  // dZ3
    const int s = s4 + 4 * j;
    float a = 0.0f;
    for (int oo = 0; oo < NO; ++oo) a += L.dy[s][oo] * P[OW4 + oo * H + o];
    L.da[s][o] = a * dact(L.z3[s][o]);
  }
  __syncthreads();
  for (int j = 0; j < H / 4; ++j) {  // dW3
    const int oo = s4 + 4 * j;
    float g = 0.0f;
    for (int s = 0; s < SB; ++s) g += L.da[s][oo] * L.h2[s][o];
    G[OW3 + oo * H + o] = g;
  }
  if (t < H) {
    float gb = 0.0f;
    for (int s = 0; s < SB; ++s) gb += L.da[s][t];
    G[OB3 + t] = gb;
  }
  {  // dZ2
    const int s = s4, u = s4 + 4;
    float a = 0.0f, c = 0.0f;
    for (int oo = 0; oo < H; ++oo) {
      const float wv = L.w3[oo * WP + o];
      a += L.da[s][oo] * wv;
      c += L.da[u][oo] * wv;
    }
    L.db[s][o] = a * dact(L.z2[s][o]);
    L.db[u][o] = c * dact(L.z2[u][o]);
  }
  __syncthreads();
  for (int j = 0; j < H / 4; ++j) {  // dW2
    const int oo = s4 + 4 * j;
    float g = 0.0f;
    for (int s = 0; s < SB; ++s) g += L.db[s][oo] * L.h1[s][o];
    G[OW2 + oo * H + o] = g;
  }
  if (t < H) {
    float gb = 0.0f;
    for (int s = 0; s < SB; ++s) gb += L.db[s][t];
    G[OB2 + t] = gb;
  }
  __syncthreads();  // da is overwritten next
  {  // dZ1
    const int s = s4, u = s4 + 4;
    float a = 0.0f, c = 0.0f;
    for (int oo = 0; oo < H; ++oo) {
      const float wv = L.w2[oo * WP + o];
      a += L.db[s][oo] * wv;
      c += L.db[u][oo] * wv;
    }
    L.da[s][o] = a * dact(L.z1[s][o]);
    L.da[u][o] = c * dact(L.z1[u][o]);
  }
  __syncthreads();
  if (t < H * NI) {  // dW1
    const int oo = t / NI, i = t % NI;
    float g = 0.0f;
    for (int s = 0; s < SB; ++s) g += L.da[s][oo] * L.x[s][i];
    G[OW1 + oo * NI + i] = g;
  }
  if (t < H) {
    float gb = 0.0f;
    for (int s = 0; s < SB; ++s) gb += L.da[s][t];
    G[OB1 + t] = gb;
  }
  if (t == 0) {
    float l = 0.0f;
    for (int q = 0; q < 256; ++q) l += L.loss[q];
    lossp[blockIdx.x] = l;
  }
}

// Fixed-order sum of the workgroup partials: 64 parameters per block of RW
// waves, wave w summing partials w, w + RW, ..., the RW sums then added by a
// fixed pairwise tree; then either the gradient is stored or Adam updates the
// parameter.  The last block sums the per-workgroup losses (strided, then a
// fixed tree).  Sixteen waves per block keep the few partials per lane in
// flight together (the sum is latency-bound: 146 blocks for 9,226 parameters).
constexpr int RW = 16;
template <bool ADAM>
__global__ __launch_bounds__(64 * RW) void k_mlp_reduce(int nwg, const float *__restrict__ partial,
                                                       const float *__restrict__ lossp, float *__restrict__ grad,
                                                       float *__restrict__ loss, float *__restrict__ P,
                                                       float *__restrict__ m, float *__restrict__ v, float lr,
                                                       float c1, float c2) {
  __shared__ float red[64 * RW];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (blockIdx.x == gridDim.x - 1) {
    float l = 0.0f;
    for (int q = threadIdx.x; q < nwg; q += 64 * RW) l += lossp[q];
    red[threadIdx.x] = l;
    __syncthreads();
    for (int st = 32 * RW; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0];
    return;
  }
  const int p = blockIdx.x * 64 + lane;
  float g = 0.0f;
  if (p < NP)
    for (int q = w; q < nwg; q += RW) g += partial[(int64_t)q * NP + p];
  red[threadIdx.x] = g;
  __syncthreads();
  for (int st = RW / 2; st > 0; st >>= 1) {  // wave w += wave w + st
    if (w < st) red[threadIdx.x] += red[threadIdx.x + 64 * st];
    __syncthreads();
  }
  if (w != 0 || p >= NP) return;
  const float gs = red[lane];
  if (!ADAM) {
    grad[p] = gs;
    return;
  }
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mm = b1 * m[p] + (1.0f - b1) * gs;
  const float vv = b2 * v[p] + (1.0f - b2) * gs * gs;
  m[p] = mm;
  v[p] = vv;
  P[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// ------------------------------------------------------------- packing
// Contraction index held by lane group g (= lane / 32) in half j of chunk c:
// the rows of a 32x32 output tile that lane group g holds, so that the output
// of one layer is the next layer's B operand without moving data.
__device__ inline int perm_k(int c, int g, int j) {
  return 32 * (c >> 1) + 16 * (c & 1) + 8 * (j >> 2) + 4 * g + (j & 3);
}

// Channel of row r of the last layer's 32-row output tile, or -1 (unused).
// Lane group g of the product holds the rows 8 (k / 4) + 4 g + k % 4 in its
// value k; rows 0-7 carry channels 0-3, rows 8-15 channels 4-7 and rows
// 16, 17 and 20, 21 channels 8, 9, so both lane groups hold all ten channels
// of their pair in values 0-9.
__host__ __device__ inline int out_channel(int r) {
  if (r < 8) return r & 3;
  if (r < 16) return 4 + (r & 3);
  if (r < 24 && (r & 3) < 2) return 8 + (r & 3);
  return -1;
}

__device__ inline void split16(double v, _Float16 &hi, _Float16 &lo) {
  hi = (_Float16)v;
  lo = (_Float16)(v - (double)hi);
}

// one thread per (operand, lane): 27 x 64 threads
__global__ void k_mlp_pack(const float *__restrict__ P, MlpNorm N, f16x8 *__restrict__ pk) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= NPK * 64) return;
  const int op = q / 64, l = q % 64, m = l & 31, g = l >> 5;
  _Float16 a[8];
  for (int j = 0; j < 8; ++j) a[j] = (_Float16)0.0f;
  if (op < PK_L2) {  // layer 1 with the input scaling x = 2 u / ext - 1 folded in
    // lane group 0: (W_hi, b_hi, W_hi, b_lo) against (u_hi, 1, u_lo, 1);
    // lane group 1: W_lo against u_hi
    const int i = 32 * op + m;
    double bs = P[OB1 + i];
    for (int k = 0; k < 3; ++k) {
      const double w = (double)P[OW1 + NI * i + k] * (2.0 / N.ext[k]);
      _Float16 hi, lo;
      split16(w, hi, lo);
      if (g == 0) a[k] = a[4 + k] = hi;
      else a[k] = lo;
      bs -= (double)P[OW1 + NI * i + k];
    }
    if (g == 0) split16(bs, a[3], a[7]);
  } else if (op < PK_L2B || (op >= PK_L3 && op < PK_L3B)) {  // W2, W3
    const int r = op < PK_L2B ? op - PK_L2 : op - PK_L3;
    const int R = r >> 2, c = r & 3, W = op < PK_L2B ? OW2 : OW3;
    for (int j = 0; j < 8; ++j) a[j] = (_Float16)P[W + H * (32 * R + m) + perm_k(c, g, j)];
  } else if (op < PK_L3 || op == PK_L3B || op == PK_L3B + 1) {  // b2, b3
    const int R = op < PK_L3 ? op - PK_L2B : op - PK_L3B;
    const int B = op < PK_L3 ? OB2 : OB3;
    if (g == 0) split16(P[B + 32 * R + m], a[0], a[1]);
  } else if (op < PK_L4B) {  // W4 scaled by sig, output row m -> channel out_channel(m)
    const int c = op - PK_L4, o = out_channel(m);
    if (o >= 0)
      for (int j = 0; j < 8; ++j) a[j] = (_Float16)((double)P[OW4 + H * o + perm_k(c, g, j)] * N.sig[o]);
  } else {  // b4 sig + mu
    const int o = out_channel(m);
    if (g == 0 && o >= 0) split16((double)P[OB4 + o] * N.sig[o] + N.mu[o], a[0], a[1]);
  }
  f16x8 v;
  for (int j = 0; j < 8; ++j) v[j] = a[j];
  pk[q] = v;
}

}  // namespace


namespace {

// The ten channels (phi_c, signed A_c, H_c) at offsets d [n][3] into out
// [n][10]; beyond the far-field switch the analytic limit as for the other
// methods.  One wave per 32 offsets.
__global__ __launch_bounds__(256) void k_mlp_points_eval(const void *__restrict__ pk, EwaldP E, int64_t n,
                                                         const double *__restrict__ d, double *__restrict__ out) {
  __shared__ f16x8 wl[64 * NPK];
  const mlpinf::Ops W = mlpinf::load_ops(pk, wl);
  const f16x8 one = mlpinf::ones();
  const int l = threadIdx.x & 63;
  const int64_t q = 32 * (((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6) + (l & 31);
  double dx = 0.0, dy = 0.0, dz = 0.0;
  if (q < n) {
    dx = d[3 * q];
    dy = d[3 * q + 1];
    dz = d[3 * q + 2];
  }
  float y[NO];
  mlpinf::forward(W, mlpinf::input((float)fabs(dx), (float)fabs(dy), (float)fabs(dz)), one, y);
  if (q >= n || l >= 32) return;
  double *o = out + NO * q;
  if (far_field10(E, dx, dy, dz, o)) return;
  const double sx = dx < 0 ? -1.0 : 1.0, sy = dy < 0 ? -1.0 : 1.0, sz = dz < 0 ? -1.0 : 1.0;
  o[0] = y[0];
  o[1] = sx * y[1];
  o[2] = sy * y[2];
  o[3] = sz * y[3];
  o[4] = y[4];
  o[5] = y[5];
  o[6] = y[6];
  o[7] = sx * sy * y[7];
  o[8] = sx * sz * y[8];
  o[9] = sy * sz * y[9];
}

// ------------------------------------------------------------- walk
// FP32 gravity walk with the surrogate's correction (BC 1 = 3P, 2 = 2P1I).
// One workgroup of 512 threads per leaf block, thread t owns cell t, the
// block's list streams through LDS once.  The network is evaluated once per
// (group of cells, list entry): the group is a node of the block-tree of
// side 2^gl cells (gl = 2: the 8 +1 nodes, 1: the 64 +2 nodes, 0: single
// cells), the largest whose cells lie within the Ewald table's half-spacing of
// its centre on every axis, so that the Taylor step below spans no more than
// the table's own (Sec. 2.2.5, second approach).  At the group centre c_g the
// offset d0 = c_g - r_node (minimum image) gives the network's ten channels at
// |d0|, unfolded to the signs of d0; a cell at delta = x - c_g then sums, with
// d = d0 + delta (the image of its group),
//   Phi -= G M (1/|d| + phi_c(d0) - A_c(d0) . delta)
//   a   -= G M (d/|d|^3 + A_c(d0) - H_c(d0) delta),
// the Newtonian part and the correction referring to the same image.  In
// 2P1I a group whose |d0_z| exceeds the far-field switch takes the analytic
// limit at every cell's d instead.  Per chunk of list entries each wave runs
// one or two batches of 32 (group, entry) pairs through the network and
// leaves their channels in LDS; after a barrier every thread sums its cell
// over the chunk.  Phi is Kahan-compensated, a summed per tile of entries.
constexpr int TW = 512;       // threads (cells) per workgroup
constexpr int TTILE = 64;     // list entries per LDS tile

struct __align__(16) TRec {
  double x, y, z;
  float m, pad;
};


template <int BC>
__global__ __launch_bounds__(TW) void k_eval_mlp_taylor(DevTree T, EwaldP E, const void *__restrict__ pk,
                                                        const int64_t *__restrict__ off,
                                                        const double4 *__restrict__ rec, float *__restrict__ phi,
                                                        float *__restrict__ acc, float negG, double tmax) {
  __shared__ f16x8 wl[64 * NPK];
  __shared__ TRec tile[TTILE];
  extern __shared__ __align__(16) float slot[];  // [pairs][TSLOT]
  const int64_t b = blockIdx.x;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, m = l & 31;
  const int64_t ncell = T.nb * 512;
  const double h = size_at(T.root_size, T.blev[b]) / 8.0;
  const int gl = mlp_group_level(h, tmax);
  const int gs = 1 << gl, ga = 8 >> gl, G = ga * ga * ga;  // group side, groups per axis, groups
  const int P = taylor_pairs(gl), C = P / G;                // pairs and entries per chunk
  const mlpinf::Ops W = mlpinf::load_ops(pk, wl);
  const f16x8 one = mlpinf::ones();
  const int64_t bx = T.bcoord[3 * b], by = T.bcoord[3 * b + 1], bz = T.bcoord[3 * b + 2];
  const double gsz = h * (double)gs;  // group edge (exact: a power-of-two multiple of h)
  // this thread's cell, its group and its offset from the group centre
  const int ci = tid, ii = ci & 7, jj = (ci >> 3) & 7, kk = ci >> 6;
  const int mg = (ii >> gl) + ga * ((jj >> gl) + ga * (kk >> gl));
  auto gcentre = [&](int g, double c[3]) {
    const int gx = g % ga, gy = (g / ga) % ga, gz = g / (ga * ga);
    if (gl == 0) {
      c[0] = centre_coord(T.org[0], 8 * bx + gx, h);
      c[1] = centre_coord(T.org[1], 8 * by + gy, h);
      c[2] = centre_coord(T.org[2], 8 * bz + gz, h);
    } else {
      c[0] = centre_coord(T.org[0], ga * bx + gx, gsz);
      c[1] = centre_coord(T.org[1], ga * by + gy, gsz);
      c[2] = centre_coord(T.org[2], ga * bz + gz, gsz);
    }
  };
  float dlx, dly, dlz;
  {
    double gc[3];
    gcentre(mg, gc);
    dlx = (float)(centre_coord(T.org[0], 8 * bx + ii, h) - gc[0]);
    dly = (float)(centre_coord(T.org[1], 8 * by + jj, h) - gc[1]);
    dlz = (float)(centre_coord(T.org[2], 8 * bz + kk, h) - gc[2]);
  }
  // the (group, entry) pairs of this lane in the network phase: batch q of
  // wave w covers pairs 32 (w + 8 q) + m, pair p = entry p / G, group p % G
  const int nbatch = P / 256;
  double pgc[2][3];
  int pent[2];
  for (int q = 0; q < 2; ++q) {
    const int p = 32 * (w + 8 * q) + m;
    pent[q] = p / G;
    gcentre(p % G, pgc[q]);
  }
  const float zfar = (float)E.zfar, fa = (float)E.far_phi_a, fb = (float)E.far_phi_b, faz = (float)E.far_az;
  float ks = 0.f, kc = 0.f, ax = 0.f, ay = 0.f, az = 0.f;
  const int64_t start = off[b], n = off[b + 1] - start;
  for (int64_t t0 = 0; t0 < n; t0 += TTILE) {
    const int mt = (int)(n - t0 < TTILE ? n - t0 : TTILE);
    __syncthreads();  // the previous tile's last chunk is consumed
    if (tid < mt) {
      const double4 r = rec[start + t0 + tid];
      tile[tid].x = r.x;
      tile[tid].y = r.y;
      tile[tid].z = r.z;
      tile[tid].m = (float)r.w;
    }
    float tx = 0.f, ty = 0.f, tz = 0.f;
    for (int j0 = 0; j0 < mt; j0 += C) {
      __syncthreads();  // tile loaded; the previous chunk's slots are consumed
      // network phase: (group, entry) pairs of this chunk; entries past the
      // tile's end repeat its last entry (their slots are never read)
      for (int q = 0; q < nbatch; ++q) {
        const int j = j0 + pent[q] < mt ? j0 + pent[q] : mt - 1;
        const TRec r = tile[j];
        const double ex = wrap_axis(pgc[q][0] - r.x, E.L[0], E.inv_L[0], 1);
        const double ey = wrap_axis(pgc[q][1] - r.y, E.L[1], E.inv_L[1], 1);
        const double ez = wrap_axis(pgc[q][2] - r.z, E.L[2], E.inv_L[2], BC == 1);
        const float dx = (float)ex, dy = (float)ey, dz = (float)ez;
        float y[NO];
        mlpinf::forward(W, mlpinf::input(fabsf(dx), fabsf(dy), fabsf(dz)), one, y);
        const float sx = ex < 0 ? -1.f : 1.f, sy = ey < 0 ? -1.f : 1.f, sz = ez < 0 ? -1.f : 1.f;
        const bool far = BC == 2 && fabs(ez) > E.zfar;
        float4 *o = reinterpret_cast<float4 *>(slot + TSLOT * (32 * (w + 8 * q) + m));
        // the two lane groups hold the same outputs: each writes half the slot
        if (l < 32) {
          o[0] = make_float4(y[0], sx * y[1], sy * y[2], sz * y[3]);
          o[1] = make_float4(y[4], y[5], y[6], sx * sy * y[7]);
        } else {
          o[2] = make_float4(sx * sz * y[8], sy * sz * y[9], dx, dy);
          o[3] = make_float4(dz, far ? 1.f : 0.f, 0.f, 0.f);
        }
      }
      __syncthreads();
      // cell phase: this thread's cell against the chunk's entries
      const int mc = mt - j0 < C ? mt - j0 : C;
      for (int j = 0; j < mc; ++j) {
        const float4 *o = reinterpret_cast<const float4 *>(slot + TSLOT * (j * G + mg));
        const float4 v0 = o[0], v1 = o[1], v2 = o[2], v3 = o[3];
        const float dx = v2.z + dlx, dy = v2.w + dly, dz = v3.x + dlz;
        const float r2 = dx * dx + dy * dy + dz * dz;
        const bool valid = r2 != 0.0f;  // the target cell itself contributes nothing
        const float inv = valid ? __builtin_amdgcn_rsqf(fmaxf(r2, 1e-30f)) : 0.0f;
        const float inv3 = inv * inv * inv;
        float ph, A0, A1, A2;
        if (BC == 2 && v3.y != 0.0f) {
          ph = fa * fabsf(dz) + fb;
          A0 = 0.0f;
          A1 = 0.0f;
          A2 = dz < 0 ? -faz : faz;
        } else {
          ph = inv + (v0.x - (v0.y * dlx + v0.z * dly + v0.w * dlz));
          A0 = dx * inv3 + (v0.y - (v1.x * dlx + v1.w * dly + v2.x * dlz));
          A1 = dy * inv3 + (v0.z - (v1.w * dlx + v1.y * dly + v2.y * dlz));
          A2 = dz * inv3 + (v0.w - (v2.x * dlx + v2.y * dly + v1.z * dlz));
        }
        const float mw = valid ? tile[j0 + j].m : 0.0f;
        const float yk = mw * ph - kc, tk = ks + yk;
        kc = (tk - ks) - yk;
        ks = tk;
        tx += mw * A0;
        ty += mw * A1;
        tz += mw * A2;
      }
    }
    ax += tx;
    ay += ty;
    az += tz;
  }
  const int64_t o = b * 512 + ci;
  phi[o] = negG * (ks - kc);
  acc[o] = negG * ax;
  acc[ncell + o] = negG * ay;
  acc[2 * ncell + o] = negG * az;
}

}  // namespace

// ------------------------------------------------------------- launchers
hipError_t launch_mlp_init(uint64_t seed, float *P, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_init, dim3((NP + 255) / 256), dim3(256), 0, st, seed, P);
  return hipGetLastError();
}

hipError_t launch_mlp_points(uint64_t seed, int64_t n, const double ext[3], double *u, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, seed, n, ext[0], ext[1],
                     ext[2], u);
  return hipGetLastError();
}

hipError_t launch_mlp_prepare(int64_t n, const double *u, const double *ser, const MlpNorm &N, float *x, float *t,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_prepare, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, u, ser, N, x, t);
  return hipGetLastError();
}

namespace {

// forward + backward of the batch [s0, s0 + batch) into the per-workgroup partials
hipError_t fwdbwd(const float *P, int64_t n, int64_t s0, int64_t batch, const float *X, const float *T,
                  float *partial, float *lossp, hipStream_t st) {
  if (batch <= 0 || batch % SB || n % SB || s0 % SB || batch > n) return hipErrorInvalidValue;
  const size_t lds = sizeof(TrainLds);
  static bool attr = false;
  if (!attr && lds > 65536) {
    hipError_t e =
        hipFuncSetAttribute((const void *)k_mlp_fwdbwd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k_mlp_fwdbwd, dim3((unsigned)(batch / SB)), dim3(256), lds, st, P, n, s0, X, T,
                     1.0f / ((float)NO * (float)batch), partial, lossp);
  return hipGetLastError();
}

constexpr unsigned reduce_blocks() { return (NP + 63) / 64 + 1; }  // + 1: the loss

}  // namespace

int64_t mlp_partials(int64_t batch) { return batch / SB; }

// ------------------------------------------------------------- fixed workspace
// Workspace of the allocation-free gradient call: the per-workgroup partial
// gradients of a batch of up to MLP_NOALLOC_MAX_BATCH samples and their
// losses, in one array that each GPU holds from library load to process exit.  Host code reaches it only through the device address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in there).
namespace {
constexpr int64_t NOALLOC_PARTIALS = MLP_NOALLOC_MAX_BATCH / SB;
constexpr int64_t NOALLOC_FLOATS = NOALLOC_PARTIALS * NP + NOALLOC_PARTIALS;
static_assert((NOALLOC_PARTIALS * NP) % 64 == 0 && NOALLOC_PARTIALS % 64 == 0, "256-byte aligned regions");
static __device__ __align__(256) float scratch[NOALLOC_FLOATS];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
float *scratch_addr[MAX_DEVICES] = {};
}  // namespace

hipError_t mlp_noalloc_workspace(int device, float **partial, float **lossp) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_addr[device]) {
    // once per device, with that device current
    hipError_t e = hipSetDevice(device);
    if (e != hipSuccess) return e;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_addr[device] = static_cast<float *>(p);
  }
  float *base = scratch_addr[device];
  *partial = base;
  *lossp = base + NOALLOC_PARTIALS * NP;
  return hipSuccess;
}

hipError_t launch_mlp_grad(const float *P, int64_t n, int64_t s0, int64_t batch, const float *X, const float *T,
                           float *partial, float *lossp, float *grad, float *loss, hipStream_t st) {
  hipError_t e = fwdbwd(P, n, s0, batch, X, T, partial, lossp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce<false>, dim3(reduce_blocks()), dim3(64 * RW), 0, st, (int)(batch / SB), partial,
                     lossp, grad, loss, (float *)nullptr, (float *)nullptr, (float *)nullptr, 0.0f, 1.0f, 1.0f);
  return hipGetLastError();
}

hipError_t launch_mlp_step(float *P, int64_t n, int64_t s0, int64_t batch, const float *X, const float *T,
                           float *partial, float *lossp, float *loss, float *m, float *v, float lr, int step,
                           hipStream_t st) {
  hipError_t e = fwdbwd(P, n, s0, batch, X, T, partial, lossp, st);
  if (e != hipSuccess) return e;
  const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(k_mlp_reduce<true>, dim3(reduce_blocks()), dim3(64 * RW), 0, st, (int)(batch / SB), partial,
                     lossp, (float *)nullptr, loss, P, m, v, lr, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mlp_pack(const float *P, const MlpNorm &N, void *pk, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_pack, dim3((NPK * 64 + 255) / 256), dim3(256), 0, st, P, N,
                     reinterpret_cast<f16x8 *>(pk));
  return hipGetLastError();
}

hipError_t launch_mlp_points_eval(const void *pk, const EwaldP &E, int64_t n, const double *d, double *out,
                                  hipStream_t st) {
  const int64_t waves = (n + 31) / 32;
  hipLaunchKernelGGL(k_mlp_points_eval, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, pk, E, n, d, out);
  return hipGetLastError();
}

size_t eval_mlp_smem(double h_max, double tmax) {
  return (size_t)taylor_pairs(mlp_group_level(h_max, tmax)) * TSLOT * sizeof(float);
}

hipError_t launch_eval_mlp(const DevTree &T, const EwaldP &E, const void *pk, const int64_t *off,
                           const double4 *rec, float *phi, float *acc, double G, double tmax, double h_max,
                           hipStream_t st) {
  dim3 grid((unsigned)T.nb), blk(TW);
  const float ng = (float)(-G);
  // dynamic LDS for the coarsest block (its groups are the smallest)
  const size_t sm = eval_mlp_smem(h_max, tmax);
  if (E.bctype == 1)
    hipLaunchKernelGGL((k_eval_mlp_taylor<1>), grid, blk, sm, st, T, E, pk, off, rec, phi, acc, ng, tmax);
  else if (E.bctype == 2)
    hipLaunchKernelGGL((k_eval_mlp_taylor<2>), grid, blk, sm, st, T, E, pk, off, rec, phi, acc, ng, tmax);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace ot
