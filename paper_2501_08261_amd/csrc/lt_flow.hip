// Learned proposal: a RealNVP-style affine-coupling flow whose conditioner
// networks run on the matrix cores (BF16 operands, FP32 accumulation), with
// FP32 master weights, Adam, and FP64 coupling arithmetic.
//
// Flow definition: coordinates whitened, u = Lw^-1 (x - mu) with Lw lower
// triangular (diag(sigma), or e.g. the Cholesky factor of a sample covariance,
// so that the network only has to model what is not Gaussian); layer l
// conditions on A_l (even l: the first floor(d/2) coordinates, odd l: the last
// floor(d/2)) and transforms B_l (the rest); conditioner h1 = relu(W1 u_A + b1),
// h2 = relu(W2 h1 + b2), o = W3 h2 + b3, s = 3 tanh(o_s / 3), t = o_t;
// y_B = u_B exp(s) + t; log q(x) = -|z|^2/2 - d/2 log 2pi + sum_l sum s_l
// - sum log diag(Lw).  Training minimises the mean negative log q of samples.
//
// Precision split: the GEMM operands (u_A, h1, h2, weights, back-propagated
// activations) are BF16, accumulation FP32; u, the coupling update, log-dets
// and log q are FP64, so that a flow whose output layer is zero is the exact
// identity and its log q the exact standardised normal density.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/lisatd.h"
#include "lt_rng.hpp"

namespace lt {
void set_error(const std::string& msg);
}

namespace lt_f {

typedef unsigned short bf16;
typedef short short4v __attribute__((ext_vector_type(4)));
typedef float float16v __attribute__((ext_vector_type(16)));

constexpr double kSMax = 3.0;
constexpr double kLog2Pi = 1.8378770664093454836;

__device__ __host__ inline bf16 to_bf16(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even (inputs are finite)
  return (bf16)(u >> 16);
}

// C[m][n] = act(sum_k A(m,k) B(k,n) + bias[n]) with A(m,k) = A[m*sAm + k*sAk],
// B(k,n) = B[k*sBk + n*sBn] (BF16), C FP32 (row stride ldc) and optional BF16
// copy Cb.  A workgroup of four wavefronts covers a 64x64 block, one 32x32
// tile per wavefront, v_mfma_f32_32x32x8bf16_1k over k in steps of 8.  Operand
// layout of the instruction (wave64): lane l supplies A[l % 32][4 (l / 32) + j]
// and B[4 (l / 32) + j][l % 32], j = 0..3, and receives
// D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32], r = 0..15.
// One 4-element fragment of a k-contiguous operand row: four consecutive BF16 values (8 bytes,
// aligned when the caller picks this path: row stride and row start multiples of 4 elements).
__device__ inline short4v frag_vec(const bf16* row, int k) {
  return *reinterpret_cast<const short4v*>(row + k);
}

// AV / BV: the A (B) operand is read as 8-byte fragments along k (sAk = 1, sAm % 4 == 0,
// aligned base; sBk = 1, sBn % 4 == 0), else element by element.  Same products in the same
// order either way.  mask (nullable): the epilogue multiplies by (mask[row][col] > 0) (the
// backward pass through a ReLU) instead of adding the bias.
template <bool AV, bool BV>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const bf16* __restrict__ A, int64_t sAm,
                                              int64_t sAk, const bf16* __restrict__ B, int64_t sBk, int64_t sBn,
                                              float* __restrict__ C, int64_t ldc, bf16* __restrict__ Cb,
                                              const float* __restrict__ bias, int relu,
                                              const float* __restrict__ mask,
                                              const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
  if (m0 >= M || n0 >= N) return;   // whole wavefront leaves together
  const int lm = lane & 31, lk = (lane >> 5) * 4;
  const int m = m0 + lm, n = n0 + lm;
  const int mr = m < M ? m : M - 1, nr = n < N ? n : N - 1;   // clamped rows for the vector reads
  float16v acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  // K in rounds of 64: the operand fragments of eight products are loaded before the first of
  // them runs (one memory latency per round instead of one per product); same product order
  constexpr int KU = 8;
  int k0 = 0;
  for (; k0 + 8 * KU <= K; k0 += 8 * KU) {
    short4v a[KU], b[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int kk = k0 + 8 * u + lk;
      if constexpr (AV) {
        a[u] = frag_vec(A + (int64_t)mr * sAm, kk);
        if (m >= M) a[u] = short4v{0, 0, 0, 0};
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) a[u][j] = m < M ? (short)A[(int64_t)m * sAm + (int64_t)(kk + j) * sAk] : (short)0;
      }
      if constexpr (BV) {
        b[u] = frag_vec(B + (int64_t)nr * sBn, kk);
        if (n >= N) b[u] = short4v{0, 0, 0, 0};
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) b[u][j] = n < N ? (short)B[(int64_t)(kk + j) * sBk + (int64_t)n * sBn] : (short)0;
      }
    }
#pragma unroll
    for (int u = 0; u < KU; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a[u], b[u], acc, 0, 0, 0);
  }
  for (; k0 < K; k0 += 8) {
    short4v a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + lk + j;
      a[j] = (k < K && m < M) ? (short)A[(int64_t)m * sAm + (int64_t)k * sAk] : (short)0;
      b[j] = (k < K && n < N) ? (short)B[(int64_t)k * sBk + (int64_t)n * sBn] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + 8 * (r >> 2) + (lane >> 5) * 4 + (r & 3);
    const int col = n0 + lm;
    if (row < M && col < N) {
      float v = acc[r];
      if (mask) {
        v = mask[(int64_t)row * ldc + col] > 0.0f ? v : 0.0f;
      } else {
        if (bias) v += bias[col];
        if (relu) v = v > 0.0f ? v : 0.0f;
      }
      C[(int64_t)row * ldc + col] = v;
      if (Cb) Cb[(int64_t)row * ldc + col] = to_bf16(v);
    }
  }
}

// Split-K partial products of the weight gradients (M, N <= a few hundred, K = the batch):
// the z-th slice of the grid sums k in [z kc, min(K, (z + 1) kc)) into part[z][M][N] with the
// instruction and operand layout of k_gemm; k_split_sum then adds the slices in order.
__global__ __launch_bounds__(256) void k_gemm_part(int M, int N, int K, int kc, const bf16* __restrict__ A,
                                                   int64_t sAm, int64_t sAk, const bf16* __restrict__ B,
                                                   int64_t sBk, int64_t sBn, float* __restrict__ part) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int m0 = blockIdx.y * 64 + (wave >> 1) * 32;
  const int n0 = blockIdx.x * 64 + (wave & 1) * 32;
  if (m0 >= M || n0 >= N) return;   // whole wavefront leaves together
  const int lm = lane & 31, lk = (lane >> 5) * 4;
  const int m = m0 + lm, n = n0 + lm;
  const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
  float16v acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  constexpr int KU = 8;
  int k0 = kb;
  for (; k0 + 8 * KU <= ke; k0 += 8 * KU) {
    short4v a[KU], b[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = k0 + 8 * u + lk + j;
        a[u][j] = m < M ? (short)A[(int64_t)m * sAm + (int64_t)k * sAk] : (short)0;
        b[u][j] = n < N ? (short)B[(int64_t)k * sBk + (int64_t)n * sBn] : (short)0;
      }
#pragma unroll
    for (int u = 0; u < KU; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a[u], b[u], acc, 0, 0, 0);
  }
  for (; k0 < ke; k0 += 8) {
    short4v a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + lk + j;
      a[j] = (k < ke && m < M) ? (short)A[(int64_t)m * sAm + (int64_t)k * sAk] : (short)0;
      b[j] = (k < ke && n < N) ? (short)B[(int64_t)k * sBk + (int64_t)n * sBn] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
  }
  float* P = part + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + 8 * (r >> 2) + (lane >> 5) * 4 + (r & 3);
    const int col = n0 + lm;
    if (row < M && col < N) P[(int64_t)row * N + col] = acc[r];
  }
}

// C[i] = sum over the slices z = 0, 1, ... of part[z][i], in that order
__global__ void k_split_sum(const float* part, int splits, int64_t mn, float* C) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= mn) return;
  float acc = part[i];
  for (int z = 1; z < splits; ++z) acc += part[(int64_t)z * mn + i];
  C[i] = acc;
}

// u (FP64 [n][d]) columns [c0, c0+w) -> BF16 [n][w]
__global__ void k_gather(const double* u, int n, int d, int c0, int w, bf16* out, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * w) return;
  const int r = i / w, c = i - r * w;
  out[i] = to_bf16((float)u[(int64_t)r * d + c0 + c]);
}

// coupling: s = S tanh(o_s / S); forward u_B <- u_B e^s + t, inverse
// u_B <- (u_B - t) e^-s; logdet += sum s (the forward log-det in both cases)
__device__ inline void couple_row(double* u, int r, int d, int b0, int nb, const float* orow, double* s_out,
                                  double* ub_in, double* logdet, int inverse) {
  double ld = 0.0;
  for (int j = 0; j < nb; ++j) {
    const double s = kSMax * tanh((double)orow[j] / kSMax);
    const double t = (double)orow[nb + j];
    double& x = u[(int64_t)r * d + b0 + j];
    if (ub_in) ub_in[(int64_t)r * nb + j] = x;
    if (s_out) s_out[(int64_t)r * nb + j] = s;
    x = inverse ? (x - t) * exp(-s) : x * exp(s) + t;
    ld += s;
  }
  logdet[r] += ld;
}

__global__ void k_couple(double* u, int n, int d, int b0, int nb, const float* o, double* s_out, double* ub_in,
                         double* logdet, int inverse, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  couple_row(u, r, d, b0, nb, o + (int64_t)r * 2 * nb, s_out, ub_in, logdet, inverse);
}

// One 32 x 32 output tile of act(A W^T + bias) for the fused coupling: A rows from LDS (BF16,
// row stride lda, K columns), W [N][K] BF16 in global memory; the same operands, products and
// product order as k_gemm, so the result is bit-identical to the unfused layer.
__device__ inline float16v tile_mma(const bf16* A, int lda, const bf16* W, int K, int N, int n0, int lane) {
  const int lm = lane & 31, lk = (lane >> 5) * 4;
  const int n = n0 + lm;
  float16v acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  constexpr int KU = 8;
  // 8-byte fragment reads: A rows sit at multiples of 4 elements of an 8-byte aligned LDS block;
  // W rows too when K is a multiple of 4 and W itself is 8-byte aligned (a uniform test)
  const bool wvec = (K % 4 == 0) && ((reinterpret_cast<uintptr_t>(W) & 7) == 0);
  int k0 = 0;
  for (; k0 + 8 * KU <= K; k0 += 8 * KU) {
    short4v a[KU], b[KU];
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const int k = k0 + 8 * u + lk;
      a[u] = *(const short4v*)(A + lm * lda + k);
      if (n < N && wvec) {
        b[u] = *(const short4v*)(W + (int64_t)n * K + k);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) b[u][j] = n < N ? (short)W[(int64_t)n * K + k + j] : (short)0;
      }
    }
#pragma unroll
    for (int u = 0; u < KU; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a[u], b[u], acc, 0, 0, 0);
  }
  for (; k0 < K; k0 += 8) {
    short4v a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + lk + j;
      a[j] = k < K ? (short)A[lm * lda + k] : (short)0;
      b[j] = (k < K && n < N) ? (short)W[(int64_t)n * K + k] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// One coupling layer applied to n rows of u (FP64 [n][d]): the rows, the layer's weights and
// the direction
struct FusedLayer {
  double* u;
  double* logdet;
  int n, a0, na, b0, nb, inverse;
  const bf16 *W1, *W2, *W3;
  const float *bias1, *bias2, *bias3;
};

// A whole coupling layer for the 32 rows of workgroup blk, when its activations need not be
// kept (sampling and log q without gradients): gather u_A, h1 = relu(u_A W1^T + b1),
// h2 = relu(h1 W2^T + b2) (BF16 in LDS, rounded where the unfused layer writes its BF16
// copies), o = h2 W3^T + b3, coupling.  LDS: u_A [32][KA], h1 and h2 [32][H] BF16,
// o [32][2 nb] FP32, s [32][nb] FP64.
constexpr int kFusedThreads = 512;   // eight wavefronts: one 32-column tile of h each at H = 256
__device__ inline void fused_layer(const FusedLayer& Ly, int blk, int d, int H, unsigned char* sm) {
  double* u = Ly.u;
  double* logdet = Ly.logdet;
  const int n = Ly.n, a0 = Ly.a0, na = Ly.na, b0 = Ly.b0, nb = Ly.nb, inverse = Ly.inverse;
  const bf16 *W1 = Ly.W1, *W2 = Ly.W2, *W3 = Ly.W3;
  const float *bias1 = Ly.bias1, *bias2 = Ly.bias2, *bias3 = Ly.bias3;
  const int KA = (na + 7) & ~7;
  bf16* uA = (bf16*)sm;
  bf16* h1 = uA + 32 * KA;
  bf16* h2 = h1 + 32 * H;
  float* o = (float*)(h2 + 32 * H);
  const int r0 = blk * 32;
  constexpr int NW = kFusedThreads / 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < 32 * KA; i += kFusedThreads) {
    const int r = i / KA, c = i - (i / KA) * KA;
    uA[i] = (r0 + r < n && c < na) ? to_bf16((float)u[(int64_t)(r0 + r) * d + a0 + c]) : (bf16)0;
  }
  __syncthreads();
  const int ntile = H / 32;
  for (int t = wave; t < ntile; t += NW) {
    const float16v acc = tile_mma(uA, KA, W1, na, H, 32 * t, lane);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r >> 2) + (lane >> 5) * 4 + (r & 3), col = 32 * t + (lane & 31);
      float v = acc[r] + bias1[col];
      v = v > 0.0f ? v : 0.0f;
      h1[row * H + col] = to_bf16(v);
    }
  }
  __syncthreads();
  for (int t = wave; t < ntile; t += NW) {
    const float16v acc = tile_mma(h1, H, W2, H, H, 32 * t, lane);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r >> 2) + (lane >> 5) * 4 + (r & 3), col = 32 * t + (lane & 31);
      float v = acc[r] + bias2[col];
      v = v > 0.0f ? v : 0.0f;
      h2[row * H + col] = to_bf16(v);
    }
  }
  __syncthreads();
  const int no = 2 * nb;
  for (int t = wave; t < (no + 31) / 32; t += NW) {
    const float16v acc = tile_mma(h2, H, W3, H, no, 32 * t, lane);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 8 * (r >> 2) + (lane >> 5) * 4 + (r & 3), col = 32 * t + (lane & 31);
      if (col < no) o[row * no + col] = acc[r] + bias3[col];
    }
  }
  __syncthreads();
  // the coupling of couple_row, one (row, j) per thread (the serial loop per row waited on a
  // load of u and an FP64 tanh and exp for each j in turn); each row's log-determinant then
  // sums its s in the order j = 0 .. nb - 1, as couple_row does
  double* sd = (double*)(o + 32 * no);   // 8-byte aligned: every block before it is
  for (int i = threadIdx.x; i < 32 * nb; i += kFusedThreads) {
    const int rr = i / nb, j = i - rr * nb, r = r0 + rr;
    if (r < n) {
      const float* orow = o + rr * no;
      const double s = kSMax * tanh((double)orow[j] / kSMax);
      const double t = (double)orow[nb + j];
      double& x = u[(int64_t)r * d + b0 + j];
      x = inverse ? (x - t) * exp(-s) : x * exp(s) + t;
      sd[i] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < 32 && r0 + (int)threadIdx.x < n) {
    double ld = 0.0;
    for (int j = 0; j < nb; ++j) ld += sd[threadIdx.x * nb + j];
    logdet[r0 + threadIdx.x] += ld;
  }
}

__global__ __launch_bounds__(kFusedThreads) void k_couple_fused(FusedLayer Ly, int d, int H,
                                                                const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  extern __shared__ __align__(16) unsigned char sm[];
  fused_layer(Ly, blockIdx.x, d, H, sm);
}

// two independent groups of rows in one launch: workgroups [0, nblk_a) run layer A on theirs,
// the others layer B (the flow move's proposals and its log q of the current positions, which
// alone fill few compute units)
__global__ __launch_bounds__(kFusedThreads) void k_couple_fused2(FusedLayer A, FusedLayer B, int nblk_a, int d, int H,
                                                                 const int* __restrict__ gate) {
  if (gate && *gate == 0) return;
  extern __shared__ __align__(16) unsigned char sm[];
  if ((int)blockIdx.x < nblk_a)
    fused_layer(A, blockIdx.x, d, H, sm);
  else
    fused_layer(B, blockIdx.x - nblk_a, d, H, sm);
}

// coupling backward: gu holds dL/dy on entry and dL/du_B on exit; writes g_o (FP32 + BF16)
__global__ void k_couple_bwd(double* gu, int n, int d, int b0, int nb, const float* o, const double* s,
                             const double* ub_in, double inv_n, float* go, bf16* gob) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  for (int j = 0; j < nb; ++j) {
    const double sj = s[(int64_t)r * nb + j], es = exp(sj);
    const double gy = gu[(int64_t)r * d + b0 + j];
    const double th = tanh((double)o[(int64_t)r * 2 * nb + j] / kSMax);
    const double gs = gy * ub_in[(int64_t)r * nb + j] * es - inv_n;   // y_B and -log|det|
    const float graw = (float)(gs * (1.0 - th * th));
    const float gt = (float)gy;
    go[(int64_t)r * 2 * nb + j] = graw;
    go[(int64_t)r * 2 * nb + nb + j] = gt;
    gob[(int64_t)r * 2 * nb + j] = to_bf16(graw);
    gob[(int64_t)r * 2 * nb + nb + j] = to_bf16(gt);
    gu[(int64_t)r * d + b0 + j] = gy * es;
  }
}

// out[c] = sum_r g[r][c]: a workgroup of 16 wavefronts takes 64 columns (each read is 64
// consecutive floats); wavefront q sums rows r = 16 i + q into eight running sums (i mod 8, so
// that eight loads are in flight), which it adds in order; the 16 wavefront sums are then added
// in order
__global__ __launch_bounds__(1024) void k_colsum(const float* g, int n, int w, float* out) {
  __shared__ float red[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  float a[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (c < w) {
    int r = wave;
    for (; r + 16 * 7 < n; r += 16 * 8)
#pragma unroll
      for (int j = 0; j < 8; ++j) a[j] += g[(int64_t)(r + 16 * j) * w + c];
    for (int j = 0; r < n; r += 16, ++j) a[j] += g[(int64_t)r * w + c];
  }
  red[wave][lane] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  __syncthreads();
  if (wave == 0 && c < w) {
    float t = 0.0f;
    for (int q = 0; q < 16; ++q) t += red[q][lane];
    out[c] = t;
  }
}

// gu[r][c0 + c] += g[r][c]
__global__ void k_scatter_add(double* gu, int n, int d, int c0, int w, const float* g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * w) return;
  const int r = i / w, c = i - r * w;
  gu[(int64_t)r * d + c0 + c] += (double)g[i];
}

// u = Lw^-1 (x[src] - mu), src = (start + r) mod n_src, by forward substitution
// (one thread per row); logdet = 0.  A diagonal Lw gives (x - mu) / sigma exactly.
__global__ void k_standardise(const double* x, int64_t n_src, int64_t start, int n, int d, const double* mu,
                              const double* Lw, double* u, double* logdet, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t src = (start + r) % n_src;
  double* ur = u + (int64_t)r * d;
  for (int i = 0; i < d; ++i) {
    double acc = 0.0;
    for (int k = 0; k < i; ++k) acc += Lw[i * d + k] * ur[k];
    ur[i] = ((x[src * d + i] - mu[i]) - acc) / Lw[i * d + i];
  }
  logdet[r] = 0.0;
}

// log q = -|u|^2/2 - d/2 log 2pi + logdet - lsig; optionally dL/dz = u / n for the mean NLL
__global__ void k_logq(const double* u, int n, int d, const double* logdet, double lsig, double* logq, double* gu,
                       double inv_n, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double q = 0.0;
  for (int c = 0; c < d; ++c) {
    const double v = u[(int64_t)r * d + c];
    q += v * v;
    if (gu) gu[(int64_t)r * d + c] = v * inv_n;
  }
  logq[r] = -0.5 * q - 0.5 * d * kLog2Pi + logdet[r] - lsig;
}

// logq += logdet - lsig (inverse pass: base density computed before it)
__global__ void k_logq_add(int n, const double* logdet, double lsig, double* logq, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  logq[r] = logq[r] + logdet[r] - lsig;
}

// x = Lw u + mu, the diagonal product and the additions rounded separately (no
// fused multiply-add), so that a diagonal Lw gives u sigma + mu exactly
__global__ void k_destandardise(const double* u, int n, int d, const double* mu, const double* Lw, double* x,
                                const int* __restrict__ gate) {
#pragma clang fp contract(off)
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * d) return;
  const int r = i / d, c = i - r * d;
  const double* ur = u + (int64_t)r * d;
  double acc = 0.0;
  for (int k = 0; k < c; ++k) acc += Lw[c * d + k] * ur[k];
  const double p = ur[c] * Lw[c * d + c];
  x[i] = (acc + p) + mu[c];
}

// u = z (the base sample)
__global__ void k_load(const double* z, int64_t count, double* u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) u[i] = z[i];
}

__global__ void k_zero(double* p, int64_t count, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0.0;
}

__global__ void k_copy(const double* src, int64_t count, double* dst, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = src[i];
}

// standard normal base samples for the proposal of walker k: Philox counter
// (step, kTagFlowZ, k, q) gives two Box-Muller pairs for coordinates 4q..4q+3
__global__ void k_base_normal(const uint64_t* step, uint32_t k0, uint32_t k1, int n, int d, double* u,
                              const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t st = (uint32_t)*step;
  for (int q = 0; 4 * q < d; ++q) {
    uint32_t c[4] = {st, lt_rng::kTagFlowZ, (uint32_t)k, (uint32_t)q};
    lt_rng::philox4x32_10(c, k0, k1);
    for (int p = 0; p < 2; ++p) {
      const double r = sqrt(-2.0 * log(lt_rng::u01(c[2 * p])));
      const double ph = 2.0 * M_PI * lt_rng::u01(c[2 * p + 1]);
      const int i0 = 4 * q + 2 * p;
      if (i0 < d) u[(int64_t)k * d + i0] = r * cos(ph);
      if (i0 + 1 < d) u[(int64_t)k * d + i0 + 1] = r * sin(ph);
    }
  }
}

// latent random walk for walker k: u <- u + sigma eps, eps standard normal from Philox counter
// (step, kTagFlowW, k, q), two Box-Muller pairs per counter as above; with
// log N(z) = -|z|^2 / 2 - (d / 2) log(2 pi) (squares summed in coordinate order):
// lq_x = logq - log N(u), lnz2 = log N(u + sigma eps)
__global__ void k_walk(const uint64_t* step, uint32_t k0, uint32_t k1, int n, int d, double sigma, double* u,
                       const double* logq, double* lq_x, double* lnz2, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t st = (uint32_t)*step;
  double e[4 * 16];
  for (int q = 0; 4 * q < d; ++q) {
    uint32_t c[4] = {st, lt_rng::kTagFlowW, (uint32_t)k, (uint32_t)q};
    lt_rng::philox4x32_10(c, k0, k1);
    for (int p = 0; p < 2; ++p) {
      const double r = sqrt(-2.0 * log(lt_rng::u01(c[2 * p])));
      const double ph = 2.0 * M_PI * lt_rng::u01(c[2 * p + 1]);
      e[4 * q + 2 * p] = r * cos(ph);
      e[4 * q + 2 * p + 1] = r * sin(ph);
    }
  }
  double z2 = 0.0, w2 = 0.0;
  for (int i = 0; i < d; ++i) {
    const double z = u[(int64_t)k * d + i];
    const double w = z + sigma * e[i];
    z2 = z2 + z * z;
    w2 = w2 + w * w;
    u[(int64_t)k * d + i] = w;
  }
  const double c0 = 0.5 * (double)d * log(2.0 * M_PI);
  lq_x[k] = logq[k] - (-0.5 * z2 - c0);
  lnz2[k] = -0.5 * w2 - c0;
}

__global__ void k_sub(double* a, const double* b, int n, const int* __restrict__ gate) {
  if (gate && *gate == 0) return;   // a sampler step without the flow move
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[k] -= b[k];
}

__global__ void k_adam(float* w, bf16* wb, const float* g, float* m, float* v, int64_t count, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  wb[i] = to_bf16(wi);
}

__global__ void k_to_bf16(const float* w, bf16* wb, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) wb[i] = to_bf16(w[i]);
}

}  // namespace lt_f

using namespace lt_f;

namespace {
struct LayerOff {
  int64_t W1, b1, W2, b2, W3, b3;
  int a0, na, b0, nb;
};
}  // namespace

struct lt_flow {
  int device = 0, d = 0, L = 0, H = 0, maxB = 0;
  // device flag read by the kernels of the sampler's flow move (nullable): 0 skips them
  const int* gate = nullptr;
  int64_t nparam = 0;
  std::vector<LayerOff> lay;
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  bf16* wb = nullptr;
  double *mu = nullptr, *Lw = nullptr;   // whitening: x = Lw u + mu, Lw [d][d] lower triangular
  double lsig = 0.0;
  int64_t t = 0;
  // per-row state (maxB rows) and per-layer activations kept for the backward pass
  double *u = nullptr, *gu = nullptr, *logdet = nullptr, *logq = nullptr, *s = nullptr, *ub = nullptr;
  double* lnz = nullptr;   // log N of the walked latent rows
  float *a1 = nullptr, *a2 = nullptr, *o = nullptr, *tmpH = nullptr, *go = nullptr, *tmpA = nullptr;
  bf16 *uA = nullptr, *h1 = nullptr, *h2 = nullptr, *gob = nullptr, *gH = nullptr;
  float* part = nullptr;   // split-K partial products of the weight gradients
  int64_t part_count = 0;
  std::vector<void*> allocs;
};

namespace {

lt_status ffail(lt_status s, const std::string& m) {
  lt::set_error(m);
  return s;
}

#define FL_HIP(call)                                                                                      \
  do {                                                                                                    \
    hipError_t e_ = (call);                                                                               \
    if (e_ != hipSuccess) return ffail(LT_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename T>
hipError_t falloc(lt_flow* f, T** p, size_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T) + 256);
  if (e == hipSuccess) {
    f->allocs.push_back(q);
    *p = (T*)q;
  }
  return e;
}

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// an operand can be read as 8-byte fragments along k: unit k stride, rows 4-element aligned
inline bool k_contiguous(const bf16* p, int64_t s_row, int64_t s_k) {
  return s_k == 1 && s_row % 4 == 0 && ((uintptr_t)p & 7) == 0;
}

void gemm(hipStream_t st, int M, int N, int K, const bf16* A, int64_t sAm, int64_t sAk, const bf16* B, int64_t sBk,
          int64_t sBn, float* C, int64_t ldc, bf16* Cb, const float* bias, int relu, const float* mask = nullptr,
          const int* gate = nullptr) {
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
  const bool av = k_contiguous(A, sAm, sAk), bv = k_contiguous(B, sBn, sBk);
  if (av && bv)
    hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, st, M, N, K, A, sAm, sAk, B, sBk, sBn, C, ldc, Cb,
                       bias, relu, mask, gate);
  else if (av)
    hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, st, M, N, K, A, sAm, sAk, B, sBk, sBn, C, ldc, Cb,
                       bias, relu, mask, gate);
  else if (bv)
    hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, st, M, N, K, A, sAm, sAk, B, sBk, sBn, C, ldc, Cb,
                       bias, relu, mask, gate);
  else
    hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, st, M, N, K, A, sAm, sAk, B, sBk, sBn, C, ldc, Cb,
                       bias, relu, mask, gate);
}

// weight gradient C[M][N] (row stride N) = sum_k A(m, k) B(k, n) over the batch K: split-K
// over slices of 128 rows of the batch (as many as the partial buffer holds), then the slices
// summed in order
void gemm_wgrad(lt_flow* f, hipStream_t st, int M, int N, int K, const bf16* A, int64_t sAm, int64_t sAk,
                const bf16* B, int64_t sBk, int64_t sBn, float* C) {
  const int64_t mn = (int64_t)M * N;
  int splits = (K + 127) / 128;
  const int64_t cap = f->part_count / mn;
  if (splits > cap) splits = (int)cap;
  if (splits < 2) {
    gemm(st, M, N, K, A, sAm, sAk, B, sBk, sBn, C, N, nullptr, nullptr, 0);
    return;
  }
  const int kc = ((K + splits - 1) / splits + 63) & ~63;
  splits = (K + kc - 1) / kc;
  dim3 grid((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64), (unsigned)splits);
  hipLaunchKernelGGL(k_gemm_part, grid, dim3(256), 0, st, M, N, K, kc, A, sAm, sAk, B, sBk, sBn, f->part);
  hipLaunchKernelGGL(k_split_sum, dim3(blocks(mn)), dim3(256), 0, st, f->part, splits, mn, C);
}

struct Slots {
  bf16 *uA, *h1, *h2;
  float *a1, *a2, *o;
  double *s, *ub;
};

Slots slots(const lt_flow* f, int l, int n) {
  const int64_t H = f->H, d = f->d;
  Slots S;
  S.uA = f->uA + l * n * d;
  S.h1 = f->h1 + l * n * H;
  S.h2 = f->h2 + l * n * H;
  S.a1 = f->a1 + l * n * H;
  S.a2 = f->a2 + l * n * H;
  S.o = f->o + l * n * 2 * d;
  S.s = f->s + l * n * d;
  S.ub = f->ub + l * n * d;
  return S;
}

// LDS of k_couple_fused for one layer (0: the layer runs unfused)
size_t fused_bytes(const lt_flow* f, const LayerOff& Lo) {
  if (f->H % 32 != 0 || f->H > 256) return 0;
  return (size_t)32 * ((Lo.na + 7) & ~7) * 2 + (size_t)2 * 32 * f->H * 2 + (size_t)32 * 2 * Lo.nb * 4 +
         (size_t)32 * Lo.nb * 8;
}

FusedLayer fused_args(const lt_flow* f, int l, double* u, double* logdet, int n, int inverse) {
  const LayerOff& Lo = f->lay[l];
  FusedLayer a;
  a.u = u;
  a.logdet = logdet;
  a.n = n;
  a.a0 = Lo.a0;
  a.na = Lo.na;
  a.b0 = Lo.b0;
  a.nb = Lo.nb;
  a.inverse = inverse;
  a.W1 = f->wb + Lo.W1;
  a.W2 = f->wb + Lo.W2;
  a.W3 = f->wb + Lo.W3;
  a.bias1 = f->w + Lo.b1;
  a.bias2 = f->w + Lo.b2;
  a.bias3 = f->w + Lo.b3;
  return a;
}

// forward (inverse = 0) or inverse pass over the n rows of f->u; logdet accumulates sum s.
// keep = false (no backward pass follows): each layer is one fused launch where it fits.
void pass(lt_flow* f, int n, int inverse, hipStream_t st, bool keep) {
  const int d = f->d, H = f->H;
  for (int q = 0; q < f->L; ++q) {
    const int l = inverse ? f->L - 1 - q : q;
    const LayerOff& Lo = f->lay[l];
    const size_t fb = keep ? 0 : fused_bytes(f, Lo);
    if (fb > 0) {
      hipLaunchKernelGGL(k_couple_fused, dim3(blocks(n, 32)), dim3(kFusedThreads), fb, st,
                         fused_args(f, l, f->u, f->logdet, n, inverse), d, H, f->gate);
      continue;
    }
    Slots S = slots(f, l, n);
    hipLaunchKernelGGL(k_gather, dim3(blocks((int64_t)n * Lo.na)), dim3(256), 0, st, f->u, n, d, Lo.a0, Lo.na, S.uA,
                       f->gate);
    gemm(st, n, H, Lo.na, S.uA, Lo.na, 1, f->wb + Lo.W1, 1, Lo.na, S.a1, H, S.h1, f->w + Lo.b1, 1, nullptr, f->gate);
    gemm(st, n, H, H, S.h1, H, 1, f->wb + Lo.W2, 1, H, S.a2, H, S.h2, f->w + Lo.b2, 1, nullptr, f->gate);
    gemm(st, n, 2 * Lo.nb, H, S.h2, H, 1, f->wb + Lo.W3, 1, H, S.o, 2 * Lo.nb, nullptr, f->w + Lo.b3, 0, nullptr,
         f->gate);
    hipLaunchKernelGGL(k_couple, dim3(blocks(n)), dim3(256), 0, st, f->u, n, d, Lo.b0, Lo.nb, S.o, S.s, S.ub,
                       f->logdet, inverse, f->gate);
  }
}

// log q of n rows x[(start + r) mod n_src] into f->logq (and dL/dz into f->gu when grad)
void logq_rows(lt_flow* f, const double* x, int64_t n_src, int64_t start, int n, bool grad, hipStream_t st) {
  hipLaunchKernelGGL(k_standardise, dim3(blocks(n, 64)), dim3(64), 0, st, x, n_src, start, n, f->d, f->mu, f->Lw,
                     f->u, f->logdet, f->gate);
  pass(f, n, 0, st, grad);
  hipLaunchKernelGGL(k_logq, dim3(blocks(n)), dim3(256), 0, st, f->u, n, f->d, f->logdet, f->lsig, f->logq,
                     grad ? f->gu : (double*)nullptr, 1.0 / n, f->gate);
}

// inverse pass from base samples already in f->u: x (FP64 [n][d]) and log q(x)
void sample_rows(lt_flow* f, int n, double* x, double* logq, hipStream_t st) {
  hipLaunchKernelGGL(k_zero, dim3(blocks(n)), dim3(256), 0, st, f->logdet, (int64_t)n, f->gate);
  hipLaunchKernelGGL(k_logq, dim3(blocks(n)), dim3(256), 0, st, f->u, n, f->d, f->logdet, 0.0, logq,
                     (double*)nullptr, 0.0, f->gate);
  pass(f, n, 1, st, false);
  hipLaunchKernelGGL(k_logq_add, dim3(blocks(n)), dim3(256), 0, st, n, f->logdet, f->lsig, logq, f->gate);
  hipLaunchKernelGGL(k_destandardise, dim3(blocks((int64_t)n * f->d)), dim3(256), 0, st, f->u, n, f->d, f->mu,
                     f->Lw, x, f->gate);
}

// backward pass of the mean NLL after logq_rows(grad = true); gradients into f->g
void backward(lt_flow* f, int n, hipStream_t s) {
  const int d = f->d, H = f->H;
  for (int l = f->L - 1; l >= 0; --l) {
    const LayerOff& Lo = f->lay[l];
    Slots S = slots(f, l, n);
    const int no = 2 * Lo.nb;
    hipLaunchKernelGGL(k_couple_bwd, dim3(blocks(n)), dim3(256), 0, s, f->gu, n, d, Lo.b0, Lo.nb, S.o, S.s, S.ub,
                       1.0 / n, f->go, f->gob);
    // dW3 = g_o^T h2, db3 = column sums of g_o
    gemm_wgrad(f, s, no, H, n, f->gob, 1, no, S.h2, H, 1, f->g + Lo.W3);
    hipLaunchKernelGGL(k_colsum, dim3(blocks(no, 64)), dim3(1024), 0, s, f->go, n, no, f->g + Lo.b3);
    // g_a2 = (g_o W3) * (h2 > 0); dW2 = g_a2^T h1
    gemm(s, n, H, no, f->gob, no, 1, f->wb + Lo.W3, H, 1, f->tmpH, H, f->gH, nullptr, 0, S.a2);
    gemm_wgrad(f, s, H, H, n, f->gH, 1, H, S.h1, H, 1, f->g + Lo.W2);
    hipLaunchKernelGGL(k_colsum, dim3(blocks(H, 64)), dim3(1024), 0, s, f->tmpH, n, H, f->g + Lo.b2);
    // g_a1 = (g_a2 W2) * (h1 > 0); dW1 = g_a1^T u_A
    gemm(s, n, H, H, f->gH, H, 1, f->wb + Lo.W2, H, 1, f->tmpH, H, f->gH, nullptr, 0, S.a1);
    gemm_wgrad(f, s, H, Lo.na, n, f->gH, 1, H, S.uA, Lo.na, 1, f->g + Lo.W1);
    hipLaunchKernelGGL(k_colsum, dim3(blocks(H, 64)), dim3(1024), 0, s, f->tmpH, n, H, f->g + Lo.b1);
    // dL/du_A += g_a1 W1
    gemm(s, n, Lo.na, H, f->gH, H, 1, f->wb + Lo.W1, Lo.na, 1, f->tmpA, Lo.na, nullptr, nullptr, 0);
    hipLaunchKernelGGL(k_scatter_add, dim3(blocks((int64_t)n * Lo.na)), dim3(256), 0, s, f->gu, n, d, Lo.a0, Lo.na,
                       f->tmpA);
  }
}

void adam(lt_flow* f, float lr, hipStream_t s) {
  f->t += 1;
  const float c1 = (float)(1.0 - std::pow(0.9, (double)f->t)), c2 = (float)(1.0 - std::pow(0.999, (double)f->t));
  hipLaunchKernelGGL(k_adam, dim3(blocks(f->nparam)), dim3(256), 0, s, f->w, f->wb, f->g, f->m, f->v, f->nparam, lr,
                     0.9f, 0.999f, 1e-8f, c1, c2);
}

lt_status check_batch(const lt_flow* f, int64_t n) {
  if (n < 1 || n > f->maxB) return ffail(LT_ERR_SHAPE, "flow batch must be in [1, max_batch]");
  return LT_OK;
}

}  // namespace

// Used by the sampler's flow move (same library, not exported).
namespace lt {
int flow_dim(const lt_flow* f) { return f->d; }
int flow_max_batch(const lt_flow* f) { return f->maxB; }
int flow_device(const lt_flow* f) { return f->device; }
// proposals y ~ q for n walkers from Philox base samples keyed by (k0, k1) at the device step counter
// gate (nullable): device flag; where it reads 0 at run time, every kernel of the call returns at once
hipError_t flow_propose(lt_flow* f, int n, const uint64_t* step, uint32_t k0, uint32_t k1, double* y, double* logq_y,
                        hipStream_t st, const int* gate) {
  f->gate = gate;
  hipLaunchKernelGGL(k_base_normal, dim3(blocks(n, 64)), dim3(64), 0, st, step, k0, k1, n, f->d, f->u, f->gate);
  sample_rows(f, n, y, logq_y, st);
  f->gate = nullptr;
  return hipGetLastError();
}
// log q of the n rows of x (FP64 [n][d]) into logq
hipError_t flow_logq(lt_flow* f, const double* x, int n, double* logq, hipStream_t st, const int* gate) {
  f->gate = gate;
  logq_rows(f, x, n, 0, n, false, st);
  hipLaunchKernelGGL(k_copy, dim3(blocks(n)), dim3(256), 0, st, f->logq, (int64_t)n, logq, f->gate);
  f->gate = nullptr;
  return hipGetLastError();
}
// flow_propose and flow_logq of the same n in one pass when the flow holds 2n rows and its
// layers run fused: the proposals in rows [0, n) of f->u, the rows of x in [n, 2n), and layer
// L-1-q of the inverse pass with layer q of the forward pass in one launch; each row sees the
// same operations as in the separate calls, so the results are the same
hipError_t flow_propose_logq(lt_flow* f, int n, const uint64_t* step, uint32_t k0, uint32_t k1, double* y,
                             double* logq_y, const double* x, double* logq_x, hipStream_t st, const int* gate) {
  const size_t fb = fused_bytes(f, f->lay[0]);
  if (2 * n > f->maxB || fb == 0) {
    hipError_t e = flow_propose(f, n, step, k0, k1, y, logq_y, st, gate);
    return e != hipSuccess ? e : flow_logq(f, x, n, logq_x, st, gate);
  }
  const int d = f->d;
  double* ux = f->u + (int64_t)n * d;
  double* ldx = f->logdet + n;
  hipLaunchKernelGGL(k_base_normal, dim3(blocks(n, 64)), dim3(64), 0, st, step, k0, k1, n, d, f->u, gate);
  hipLaunchKernelGGL(k_zero, dim3(blocks(n)), dim3(256), 0, st, f->logdet, (int64_t)n, gate);
  hipLaunchKernelGGL(k_logq, dim3(blocks(n)), dim3(256), 0, st, f->u, n, d, f->logdet, 0.0, logq_y,
                     (double*)nullptr, 0.0, gate);
  hipLaunchKernelGGL(k_standardise, dim3(blocks(n, 64)), dim3(64), 0, st, x, (int64_t)n, (int64_t)0, n, d, f->mu,
                     f->Lw, ux, ldx, gate);
  const unsigned nblk = blocks(n, 32);
  for (int q = 0; q < f->L; ++q)
    hipLaunchKernelGGL(k_couple_fused2, dim3(2 * nblk), dim3(kFusedThreads), fb, st,
                       fused_args(f, f->L - 1 - q, f->u, f->logdet, n, 1), fused_args(f, q, ux, ldx, n, 0),
                       (int)nblk, d, f->H, gate);
  hipLaunchKernelGGL(k_logq_add, dim3(blocks(n)), dim3(256), 0, st, n, f->logdet, f->lsig, logq_y, gate);
  hipLaunchKernelGGL(k_destandardise, dim3(blocks((int64_t)n * d)), dim3(256), 0, st, f->u, n, d, f->mu, f->Lw, y,
                     gate);
  hipLaunchKernelGGL(k_logq, dim3(blocks(n)), dim3(256), 0, st, ux, n, d, ldx, f->lsig, logq_x, (double*)nullptr,
                     1.0 / n, gate);
  return hipGetLastError();
}
// latent random walk from the rows of x: z = f(x), y = f^-1(z + sigma eps);
// lq_x = log q(x) - log N(z), lq_y = log q(y) - log N(z + sigma eps)
hipError_t flow_walk(lt_flow* f, const double* x, int n, const uint64_t* step, uint32_t k0, uint32_t k1, double sigma,
                     double* y, double* lq_y, double* lq_x, hipStream_t st, const int* gate) {
  f->gate = gate;
  logq_rows(f, x, n, 0, n, false, st);
  hipLaunchKernelGGL(k_walk, dim3(blocks(n, 64)), dim3(64), 0, st, step, k0, k1, n, f->d, sigma, f->u, f->logq, lq_x,
                     f->lnz, f->gate);
  sample_rows(f, n, y, lq_y, st);
  hipLaunchKernelGGL(k_sub, dim3(blocks(n)), dim3(256), 0, st, lq_y, f->lnz, n, f->gate);
  f->gate = nullptr;
  return hipGetLastError();
}
}  // namespace lt

extern "C" {

lt_status lt_flow_create(int hip_device, int dim, int n_layers, int hidden, int max_batch, lt_flow** out) {
  if (!out) return ffail(LT_ERR_NULL, "null output");
  if (dim < 2 || dim > 64 || n_layers < 1 || n_layers > 32 || hidden < 8 || hidden > 4096 || hidden % 8 ||
      max_batch < 1 || max_batch > (1 << 20))
    return ffail(LT_ERR_SHAPE, "flow dimensions: 2 <= dim <= 64, 1 <= layers <= 32, hidden in [8, 4096] and a "
                               "multiple of 8, 1 <= max_batch <= 2^20");
  FL_HIP(hipSetDevice(hip_device));
  lt_flow* f = new lt_flow();
  f->device = hip_device;
  f->d = dim;
  f->L = n_layers;
  f->H = hidden;
  f->maxB = max_batch;
  int64_t off = 0;
  const int da = dim / 2;
  for (int l = 0; l < n_layers; ++l) {
    LayerOff Lo;
    Lo.na = da;
    Lo.nb = dim - da;
    Lo.a0 = (l % 2 == 0) ? 0 : dim - da;
    Lo.b0 = (l % 2 == 0) ? da : 0;
    Lo.W1 = off; off += (int64_t)hidden * Lo.na;
    Lo.b1 = off; off += hidden;
    Lo.W2 = off; off += (int64_t)hidden * hidden;
    Lo.b2 = off; off += hidden;
    Lo.W3 = off; off += (int64_t)2 * Lo.nb * hidden;
    Lo.b3 = off; off += 2 * Lo.nb;
    f->lay.push_back(Lo);
  }
  f->nparam = off;
  const int64_t B = max_batch, H = hidden, L = n_layers;
  hipError_t e = hipSuccess;
#define FA(ptr, cnt) \
  if (e == hipSuccess) e = falloc(f, &f->ptr, (size_t)(cnt))
  FA(w, off); FA(g, off); FA(m, off); FA(v, off); FA(wb, off);
  FA(mu, dim); FA(Lw, (int64_t)dim * dim);
  FA(u, B * dim); FA(gu, B * dim); FA(logdet, B); FA(logq, B); FA(lnz, B);
  FA(a1, L * B * H); FA(a2, L * B * H); FA(o, L * B * 2 * dim); FA(s, L * B * dim); FA(ub, L * B * dim);
  FA(uA, L * B * dim); FA(h1, L * B * H); FA(h2, L * B * H);
  FA(tmpH, B * H); FA(go, B * 2 * dim); FA(gob, B * 2 * dim); FA(gH, B * H); FA(tmpA, B * dim);
  // split-K partials: up to 16 slices of the largest weight matrix, at most 64 MiB
  {
    const int64_t mx = H * std::max<int64_t>(H, 2 * dim);
    int64_t sl = std::min<int64_t>(16, ((B + 127) / 128));
    while (sl > 1 && sl * mx * 4 > ((int64_t)64 << 20)) --sl;
    f->part_count = sl > 1 ? sl * mx : 0;
    if (f->part_count) FA(part, f->part_count);
  }
#undef FA
  if (e != hipSuccess) {
    lt_flow_destroy(f);
    return ffail(LT_ERR_DEVICE, std::string("flow allocation: ") + hipGetErrorString(e));
  }
  std::vector<double> eye((size_t)dim * dim, 0.0), zero(dim, 0.0);
  for (int i = 0; i < dim; ++i) eye[(size_t)i * dim + i] = 1.0;
  std::vector<float> zf(off, 0.0f);
  if (hipMemcpy(f->mu, zero.data(), dim * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(f->Lw, eye.data(), eye.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(f->w, zf.data(), off * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(f->m, zf.data(), off * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(f->v, zf.data(), off * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    lt_flow_destroy(f);
    return ffail(LT_ERR_DEVICE, "flow initialisation copies");
  }
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks(off)), dim3(256), 0, 0, f->w, f->wb, off);
  if (hipDeviceSynchronize() != hipSuccess) {
    lt_flow_destroy(f);
    return ffail(LT_ERR_DEVICE, "flow initialisation");
  }
  *out = f;
  return LT_OK;
}

lt_status lt_flow_destroy(lt_flow* f) {
  if (!f) return ffail(LT_ERR_NULL, "null flow");
  (void)hipSetDevice(f->device);
  (void)hipDeviceSynchronize();
  for (void* p : f->allocs) (void)hipFree(p);
  delete f;
  return LT_OK;
}

int64_t lt_flow_num_params(const lt_flow* f) { return f ? f->nparam : -1; }

static lt_status set_whitening(lt_flow* f, const double* mu, const double* L, bool diagonal) {
  const int d = f->d;
  std::vector<double> W((size_t)d * d, 0.0);
  double lsig = 0.0;
  for (int i = 0; i < d; ++i) {
    const double di = diagonal ? L[i] : L[(size_t)i * d + i];
    if (!(di > 0.0) || !std::isfinite(di) || !std::isfinite(mu[i]))
      return ffail(LT_ERR_CONFIG, "mu must be finite and the whitening diagonal positive");
    lsig += std::log(di);
    W[(size_t)i * d + i] = di;
    if (!diagonal)
      for (int k = 0; k < i; ++k) {
        if (!std::isfinite(L[(size_t)i * d + k])) return ffail(LT_ERR_CONFIG, "non-finite whitening matrix");
        W[(size_t)i * d + k] = L[(size_t)i * d + k];
      }
  }
  FL_HIP(hipSetDevice(f->device));
  FL_HIP(hipDeviceSynchronize());
  FL_HIP(hipMemcpy(f->mu, mu, d * sizeof(double), hipMemcpyHostToDevice));
  FL_HIP(hipMemcpy(f->Lw, W.data(), W.size() * sizeof(double), hipMemcpyHostToDevice));
  f->lsig = lsig;
  return LT_OK;
}

lt_status lt_flow_set_params(lt_flow* f, const float* params, const double* mu, const double* sigma) {
  if (!f || !params || !mu || !sigma) return ffail(LT_ERR_NULL, "null argument");
  for (int64_t i = 0; i < f->nparam; ++i)
    if (!std::isfinite(params[i])) return ffail(LT_ERR_CONFIG, "non-finite flow parameter");
  lt_status st = set_whitening(f, mu, sigma, true);
  if (st) return st;
  FL_HIP(hipMemcpy(f->w, params, f->nparam * sizeof(float), hipMemcpyHostToDevice));
  std::vector<float> zf(f->nparam, 0.0f);
  FL_HIP(hipMemcpy(f->m, zf.data(), f->nparam * sizeof(float), hipMemcpyHostToDevice));
  FL_HIP(hipMemcpy(f->v, zf.data(), f->nparam * sizeof(float), hipMemcpyHostToDevice));
  f->t = 0;
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks(f->nparam)), dim3(256), 0, 0, f->w, f->wb, f->nparam);
  FL_HIP(hipDeviceSynchronize());
  return LT_OK;
}

lt_status lt_flow_set_whitening(lt_flow* f, const double* mu, const double* L) {
  if (!f || !mu || !L) return ffail(LT_ERR_NULL, "null argument");
  return set_whitening(f, mu, L, false);
}

lt_status lt_flow_get_params(lt_flow* f, float* params) {
  if (!f || !params) return ffail(LT_ERR_NULL, "null argument");
  FL_HIP(hipSetDevice(f->device));
  FL_HIP(hipDeviceSynchronize());
  FL_HIP(hipMemcpy(params, f->w, f->nparam * sizeof(float), hipMemcpyDeviceToHost));
  return LT_OK;
}

lt_status lt_flow_log_prob(lt_flow* f, const double* x, int64_t n, double* logq, void* stream) {
  if (!f || !x || !logq) return ffail(LT_ERR_NULL, "null argument");
  lt_status st = check_batch(f, n);
  if (st) return st;
  FL_HIP(hipSetDevice(f->device));
  hipStream_t s = (hipStream_t)stream;
  logq_rows(f, x, n, 0, (int)n, false, s);
  hipLaunchKernelGGL(k_copy, dim3(blocks(n)), dim3(256), 0, s, f->logq, n, logq, f->gate);
  FL_HIP(hipGetLastError());
  return LT_OK;
}

lt_status lt_flow_sample(lt_flow* f, const double* z, int64_t n, double* x, double* logq, void* stream) {
  if (!f || !z || !x || !logq) return ffail(LT_ERR_NULL, "null argument");
  lt_status st = check_batch(f, n);
  if (st) return st;
  FL_HIP(hipSetDevice(f->device));
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_load, dim3(blocks(n * f->d)), dim3(256), 0, s, z, n * f->d, f->u);
  sample_rows(f, (int)n, x, logq, s);
  FL_HIP(hipGetLastError());
  return LT_OK;
}

lt_status lt_flow_loss_grad(lt_flow* f, const double* x, int64_t n, double* logq, float* grad) {
  if (!f || !x) return ffail(LT_ERR_NULL, "null argument");
  lt_status st = check_batch(f, n);
  if (st) return st;
  FL_HIP(hipSetDevice(f->device));
  logq_rows(f, x, n, 0, (int)n, true, 0);
  backward(f, (int)n, 0);
  FL_HIP(hipGetLastError());
  FL_HIP(hipDeviceSynchronize());
  if (logq) FL_HIP(hipMemcpy(logq, f->logq, n * sizeof(double), hipMemcpyDeviceToHost));
  if (grad) FL_HIP(hipMemcpy(grad, f->g, f->nparam * sizeof(float), hipMemcpyDeviceToHost));
  return LT_OK;
}

lt_status lt_flow_train(lt_flow* f, const double* x, int64_t n, int steps, int batch, double lr, void* stream) {
  if (!f || !x) return ffail(LT_ERR_NULL, "null argument");
  if (n < 1 || steps < 0) return ffail(LT_ERR_SHAPE, "training sizes");
  lt_status st = check_batch(f, batch);
  if (st) return st;
  if (!(lr > 0.0) || !std::isfinite(lr)) return ffail(LT_ERR_CONFIG, "lr must be positive");
  FL_HIP(hipSetDevice(f->device));
  hipStream_t s = (hipStream_t)stream;
  for (int it = 0; it < steps; ++it) {
    const int64_t start = ((int64_t)it * batch) % n;
    logq_rows(f, x, n, start, batch, true, s);
    backward(f, batch, s);
    adam(f, (float)lr, s);
  }
  FL_HIP(hipGetLastError());
  return LT_OK;
}

}  // extern "C"
