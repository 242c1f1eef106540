// Learned warm start: a small MLP (BF16 operands, FP32 accumulate) trained
// and evaluated with hand-written MFMA GEMMs on gfx950.
//
// Layers: h_0 = x, h_{l+1} = relu(h_l W_l + b_l) for hidden layers, output
// y = h_L W_L + b_L.  Weights live as FP32 masters (Adam state beside them)
// and BF16 copies used by the GEMMs; activations are stored in BF16, the
// pre-activation mask in the ReLU backward comes from the stored activation.
//
// GEMM: C[M x N] = op(A)[M x K] op(B)[K x N] with op = transpose or not,
// row-major storage, zero-filled edges (no padding required).  Block tile
// 128 x 128 x 64, 256 threads = 4 wavefronts of 64 x 64 (2 x 2 tiles of the
// 32 x 32 x 16 BF16 MFMA).  Operand layout of v_mfma_f32_32x32x16_bf16: lane l
// holds row (l mod 32) of A and column (l mod 32) of B for k in
// [8 (l div 32), 8 (l div 32) + 8); accumulator register v of lane l is
// C[8 (v div 4) + 4 (l div 32) + (v mod 4)][l mod 32].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "../../include/gridplan.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BN = 128, BK = 64;
constexpr int LDA = BK + 8;  // LDS row pitch (bf16): 144 bytes, keeps 16-byte alignment

__device__ __forceinline__ __bf16 to_bf16(float v) { return (__bf16)v; }

enum Epi { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2 };

struct GemmArgs {
  const __bf16* A;
  const __bf16* B;
  float* Cf;         // FP32 output [M x N] (nullable)
  __bf16* Cb;        // BF16 output [M x N] (nullable)
  const float* bias;
  int M, N, K;       // C = op(A) op(B), k in [0, K)
  int lda, ldb;      // row strides of A and B as stored
  int Ka, Kb;        // entries of A / B with k >= Ka / Kb read as zero
  int epi, accumulate;
  int vecA, vecB;    // 1: stage 8 contiguous elements per 16-byte load
  int vecC;          // 1: BF16 output written as 16-byte segments through LDS
};

typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

// one 8-element chunk of a staged operand: 8 bf16 in registers
struct Chunk {
  u16x8 v;
};

__device__ __forceinline__ unsigned short bits(__bf16 x) { return __builtin_bit_cast(unsigned short, x); }
__device__ __forceinline__ __bf16 frombits(unsigned short u) { return __builtin_bit_cast(__bf16, u); }

// Operand tiles in LDS are [row][k] (row = m for A, n for B), BK k per
// row.  A tile of R rows has R*BK/8 chunks of 8 k; thread t stages chunks
// t, t + 256, ...  For a "k-contiguous" operand (A not transposed, B
// transposed) a chunk is 8 consecutive k of one row; otherwise it is 8
// consecutive rows at one k (stored transposed into LDS).
template <int R, bool KCONT>
__device__ __forceinline__ void load_chunks(const __bf16* __restrict__ P, int ld, int row0, int nrows, int k0,
                                            int kvalid, bool vec, Chunk (&c)[R * BK / 8 / 256]) {
  constexpr int NC = R * BK / 8 / 256;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int e = (int)threadIdx.x + 256 * q;
    if (KCONT) {
      const int r = e / (BK / 8), kq = (e % (BK / 8)) * 8;
      const int gr = row0 + r, gk = k0 + kq;
      if (vec) {
        if (gr < nrows && gk < kvalid) c[q].v = *reinterpret_cast<const u16x8*>(P + (int64_t)gr * ld + gk);
        else c[q].v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
          c[q].v[i] = (gr < nrows && gk + i < kvalid) ? bits(P[(int64_t)gr * ld + gk + i]) : (unsigned short)0;
      }
    } else {
      const int k = e / (R / 8), rq = (e % (R / 8)) * 8;
      const int gr = row0 + rq, gk = k0 + k;
      if (vec) {
        if (gr < nrows && gk < kvalid) c[q].v = *reinterpret_cast<const u16x8*>(P + (int64_t)gk * ld + gr);
        else c[q].v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i)
          c[q].v[i] = (gr + i < nrows && gk < kvalid) ? bits(P[(int64_t)gk * ld + gr + i]) : (unsigned short)0;
      }
    }
  }
}

template <int R, bool KCONT>
__device__ __forceinline__ void store_chunks(__bf16* __restrict__ S, const Chunk (&c)[R * BK / 8 / 256]) {
  constexpr int NC = R * BK / 8 / 256;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int e = (int)threadIdx.x + 256 * q;
    if (KCONT) {
      const int r = e / (BK / 8), kq = (e % (BK / 8)) * 8;
      *reinterpret_cast<u16x8*>(S + r * LDA + kq) = c[q].v;
    } else {
      const int k = e / (R / 8), rq = (e % (R / 8)) * 8;
#pragma unroll
      for (int i = 0; i < 8; ++i) S[(rq + i) * LDA + k] = frombits(c[q].v[i]);
    }
  }
}

// C = op(A) op(B) (+ bias, relu), BF16 operands, FP32 accumulation on the
// 32x32x16 MFMA.  Block tile BM x 128 x 64 with 4 wavefronts in 2 x 2, each
// owning (BM/2) x 64 of C; the next K tile is fetched into registers while
// the current one is multiplied.
//
// Tile order: the grid is 1-D and workgroups go to the 8 XCDs round-robin
// (workgroup b to XCD b mod 8), so XCD x is given the contiguous range of
// tiles [x q + min(x, r), ...) (q = tiles / 8, r = tiles mod 8) in row-panel
// order: the column tiles of one row panel of A run on one XCD at about the
// same time and share its L2, and A is fetched from HBM about once.
//
// BF16 output (hidden layers) is staged through LDS after the last K tile and
// written as 16-byte row segments; FP32 output is written from the
// accumulators directly.
template <int BM, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  static_assert(BM == 64 || BM == 128, "BM");
  constexpr int MI = BM / 64;  // 32-row MFMA tiles per wave along m
  constexpr int CP = BN + 8;   // row pitch of the staged C tile (bf16)
  static_assert(BM * CP <= (BM + BN) * LDA, "the C tile fits in the operand tiles");
  __shared__ __attribute__((aligned(16))) __bf16 smem[(BM + BN) * LDA];
  __bf16* As = smem;
  __bf16* Bs = smem + BM * LDA;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gn = (g.N + BN - 1) / BN;
  const int tiles = gn * ((g.M + BM - 1) / BM);
  const int xcd = (int)blockIdx.x & 7, q = tiles >> 3, r8 = tiles & 7;
  const int tile = xcd * q + min(xcd, r8) + ((int)blockIdx.x >> 3);
  const int m0 = (tile / gn) * BM, n0 = (tile % gn) * BN;
  const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * 64;
  f32x16 acc[MI][2];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.f;

  Chunk ca[BM * BK / 8 / 256], cb[BN * BK / 8 / 256];
  load_chunks<BM, !TA>(g.A, g.lda, m0, g.M, 0, g.Ka, g.vecA, ca);
  load_chunks<BN, TB>(g.B, g.ldb, n0, g.N, 0, g.Kb, g.vecB, cb);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    store_chunks<BM, !TA>(As, ca);
    store_chunks<BN, TB>(Bs, cb);
    __syncthreads();
    if (k0 + BK < g.K) {  // prefetch the next K tile while this one is used
      load_chunks<BM, !TA>(g.A, g.lda, m0, g.M, k0 + BK, g.Ka, g.vecA, ca);
      load_chunks<BN, TB>(g.B, g.ldb, n0, g.N, k0 + BK, g.Kb, g.vecB, cb);
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      const int kq = ks + 8 * (lane >> 5);
      bf16x8 af[MI], bfr[2];
#pragma unroll
      for (int i = 0; i < MI; ++i)
        af[i] = *reinterpret_cast<const bf16x8*>(&As[(wm + 32 * i + (lane & 31)) * LDA + kq]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bfr[j] = *reinterpret_cast<const bf16x8*>(&Bs[(wn + 32 * j + (lane & 31)) * LDA + kq]);
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  if (g.Cb && !g.Cf && g.vecC) {
    // the loop ended on a barrier, so the operand tiles are free for C
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int cl = wn + 32 * j + (lane & 31);
        const float bv = (g.epi != EPI_NONE && n0 + cl < g.N) ? g.bias[n0 + cl] : 0.f;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int rl = wm + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
          float r = acc[i][j][v] + bv;
          if (g.epi == EPI_BIAS_RELU) r = fmaxf(r, 0.f);
          smem[rl * CP + cl] = to_bf16(r);
        }
      }
    __syncthreads();
    // N is a multiple of 8, so a segment starting inside the matrix ends inside it
#pragma unroll
    for (int c = 0; c < BM * BN / 8 / 256; ++c) {
      const int e = (int)threadIdx.x + 256 * c;
      const int rl = e / (BN / 8), cl = (e % (BN / 8)) * 8;
      if (m0 + rl < g.M && n0 + cl < g.N)
        *reinterpret_cast<u16x8*>(g.Cb + (int64_t)(m0 + rl) * g.N + n0 + cl) =
            *reinterpret_cast<const u16x8*>(&smem[rl * CP + cl]);
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        const int col = n0 + wn + 32 * j + (lane & 31);
        if (row < g.M && col < g.N) {
          float r = acc[i][j][v];
          if (g.epi != EPI_NONE) r += g.bias[col];
          if (g.epi == EPI_BIAS_RELU) r = fmaxf(r, 0.f);
          const int64_t o = (int64_t)row * g.N + col;
          if (g.Cf) g.Cf[o] = g.accumulate ? g.Cf[o] + r : r;
          if (g.Cb) g.Cb[o] = to_bf16(r);
        }
      }
}

// Wt [N x ldt] = bf16(W [K x N])^T, zero in columns K..ldt-1
__global__ void k_transpose_bf16(const float* __restrict__ W, __bf16* __restrict__ Wt, int K, int N, int ldt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)N * ldt) return;
  const int n = (int)(i / ldt), k = (int)(i - (int64_t)n * ldt);
  Wt[i] = to_bf16(k < K ? W[(int64_t)k * N + n] : 0.f);
}

__global__ void k_cast_bf16(const float* __restrict__ x, __bf16* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

// network input: Y [rows x npad] = bf16((X - mu[c]) * isd[c]) for c < ncol
// (no standardisation when mu is null), zero in the padding columns
__global__ void k_cast_input(const float* __restrict__ x, __bf16* __restrict__ y, int64_t rows, int ncol, int npad,
                             const float* __restrict__ mu, const float* __restrict__ isd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * npad) return;
  const int64_t r = i / npad;
  const int c = (int)(i - r * npad);
  float v = 0.f;
  if (c < ncol) {
    v = x[r * ncol + c];
    if (mu) v = (v - mu[c]) * isd[c];
  }
  y[i] = to_bf16(v);
}

// network output back in target units: Y = Z * sd[c] + mu[c]
__global__ void k_unscale(const float* __restrict__ Z, float* __restrict__ Y, int64_t n, int ncol,
                          const float* __restrict__ mu, const float* __restrict__ sd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % ncol);
  Y[i] = Z[i] * sd[c] + mu[c];
}

// column sums and sums of squares over one chunk of rows (FP64)
__global__ void k_colstats_part(const float* __restrict__ X, int64_t rows, int ncol, int64_t chunk,
                                double* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  const int64_t r0 = (int64_t)blockIdx.y * chunk, r1 = r0 + chunk < rows ? r0 + chunk : rows;
  double s = 0.0, q = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double v = X[r * ncol + c];
    s += v;
    q += v * v;
  }
  part[(int64_t)(2 * blockIdx.y) * ncol + c] = s;
  part[(int64_t)(2 * blockIdx.y + 1) * ncol + c] = q;
}

// mean and standard deviation per column (chunks summed in order); a column
// with (numerically) no spread keeps sd = 1 and is only centred
__global__ void k_colstats_final(const double* __restrict__ part, int nchunk, int ncol, int64_t rows,
                                 float* __restrict__ mu, float* __restrict__ sd, float* __restrict__ isd) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  double s = 0.0, q = 0.0;
  for (int k = 0; k < nchunk; ++k) {
    s += part[(int64_t)(2 * k) * ncol + c];
    q += part[(int64_t)(2 * k + 1) * ncol + c];
  }
  const double m = s / (double)rows;
  const double v = fmax(q / (double)rows - m * m, 0.0);
  double d = sqrt(v);
  if (!(d > 1e-6 * (1.0 + fabs(m)))) d = 1.0;
  mu[c] = (float)m;
  sd[c] = (float)d;
  isd[c] = 1.f / (float)d;
}

// dY = (2 / count) (Y - T') per element with T' = (T - mu[c]) * isd[c] when
// the targets are standardised (mu non-null); loss partials per block (FP64)
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, float* __restrict__ dY,
                      __bf16* __restrict__ dYb, double* __restrict__ part, int64_t n, double scale, int ncol,
                      const float* __restrict__ mu, const float* __restrict__ isd) {
  __shared__ double sh[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (i < n) {
    float t = T[i];
    if (mu) {
      const int c = (int)(i % ncol);
      t = (t - mu[c]) * isd[c];
    }
    const float d = Y[i] - t;
    l = (double)d * d;
    const float g = (float)(2.0 * scale) * d;
    dY[i] = g;
    dYb[i] = to_bf16(g);
  }
  sh[threadIdx.x] = l;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// ReLU backward through a stored BF16 activation: g *= (h > 0); BF16 copy
__global__ void k_relu_bwd(float* __restrict__ g, const __bf16* __restrict__ h, __bf16* __restrict__ gb,
                           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const float v = ((float)h[i] > 0.f) ? g[i] : 0.f;
    g[i] = v;
    gb[i] = to_bf16(v);
  }
}

// bias gradient: column sums of G [M x N] in a fixed order
__global__ void k_colsum(const float* __restrict__ G, float* __restrict__ out, int M, int N) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  double s = 0.0;
  for (int r = 0; r < M; ++r) s += G[(int64_t)r * N + c];
  out[c] = (float)s;
}

// Adam on FP32 masters (bias-corrected), then the BF16 copy
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, __bf16* __restrict__ wb, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = to_bf16(wi);
}

struct MlpError {
  int code;
  std::string msg;
};

[[noreturn]] void mfail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  throw MlpError{code, buf};
}

#define MCHK(expr)                                                                       \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) mfail(GP_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

template <class T>
struct Buf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t c) {
    if (c <= n && p) return;
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
    if (!c) return;
    hipError_t e = hipMalloc((void**)&p, c * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      mfail(e == hipErrorOutOfMemory ? GP_ENOMEM : GP_EHIP, "hipMalloc failed");
    }
    n = c;
  }
  ~Buf() {
    if (p) (void)hipFree(p);
  }
};

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

// C [M x N] = op(A) op(B).  A: ta ? [K x M] (stride lda) : [M x K] (stride
// lda); B: tb ? [N x K] : [K x N] (stride ldb).  Entries at k >= Ka of A and
// k >= Kb of B are read as zero (padding columns of A may hold anything
// finite only if Kb bounds them).
void launch_gemm(bool ta, bool tb, const __bf16* A, int lda, int Ka, const __bf16* B, int ldb, int Kb, float* Cf,
                 __bf16* Cb, const float* bias, int M, int N, int K, int epi, int accumulate, hipStream_t st) {
  GemmArgs g{A, B, Cf, Cb, bias, M, N, K, lda, ldb, Ka, Kb, epi, accumulate, 0, 0, 0};
  // 16-byte staging needs every chunk to start on a multiple of 8 elements
  // of an aligned base and to lie wholly inside or outside the valid range
  g.vecA = aligned16(A) && lda % 8 == 0 && (ta ? M % 8 == 0 : Ka % 8 == 0);
  g.vecB = aligned16(B) && ldb % 8 == 0 && (tb ? Kb % 8 == 0 : N % 8 == 0);
  g.vecC = Cb && aligned16(Cb) && N % 8 == 0;
  const int gn = (N + BN - 1) / BN;
  const bool small = (int64_t)gn * ((M + 127) / 128) < 512;  // fill the CUs with 64-row tiles
  if ((int64_t)gn * ((M + 63) / 64) > INT32_MAX) mfail(GP_EINVAL, "GEMM of %d x %d has too many tiles", M, N);
#define GEMM_(BMv)                                                                                 \
  {                                                                                                \
    dim3 grid(gn * ((M + BMv - 1) / BMv));                                                         \
    if (!ta && !tb) hipLaunchKernelGGL((k_gemm<BMv, false, false>), grid, dim3(256), 0, st, g);     \
    else if (!ta && tb) hipLaunchKernelGGL((k_gemm<BMv, false, true>), grid, dim3(256), 0, st, g);  \
    else if (ta && !tb) hipLaunchKernelGGL((k_gemm<BMv, true, false>), grid, dim3(256), 0, st, g);  \
    else hipLaunchKernelGGL((k_gemm<BMv, true, true>), grid, dim3(256), 0, st, g);                  \
  }
  if (small) GEMM_(64) else GEMM_(128)
#undef GEMM_
  MCHK(hipGetLastError());
}

int nblk(int64_t n, int b = 256) { return (int)((n + b - 1) / b); }

// Scratch of the allocation-free forward pass (mlp_forward_noalloc): two BF16
// activation buffers that the layers alternate between.  One copy per GPU,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in; kernels get the device address taken once per device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// the device address of the current device's scratch (taken on first use)
void* scratch_address() {
  int dev = 0;
  MCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) mfail(GP_EINVAL, "device %d beyond the %d the library tracks", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      mfail(GP_EHIP, "hipGetSymbolAddress of the forward scratch failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

struct gp_mlp {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::vector<int> dims;  // n_in, width..., n_out
  int L = 0;              // number of linear layers
  int n_pad = 0;          // input row stride: n_in rounded up to 32 (zero columns)
  std::vector<int64_t> woff, boff;  // offsets into the flat parameter vector
  int64_t nparam = 0;
  Buf<float> w, g, m, v;  // FP32 masters, gradients, Adam moments
  Buf<__bf16> wb;         // BF16 copy (weights only; biases stay FP32)
  // BF16 transposed copy for the forward pass: layer l as [out x in_l]
  // (row stride n_pad for layer 0, zero padding), so both forward operands
  // are staged k-contiguous with 16-byte loads and stores
  Buf<__bf16> wbt;
  std::vector<int64_t> wtoff;
  int64_t step = 0;
  // activations for a batch
  int64_t cap_rows = 0;
  std::vector<Buf<__bf16>> act;  // act[l]: input of layer l, [rows x width_l] BF16 (layer 0: n_pad)
  Buf<float> out, dy;            // [rows x n_out] FP32
  Buf<float> gf;                 // FP32 gradient wrt a hidden activation (largest width)
  Buf<__bf16> gb0, gb1;          // BF16 gradients (ping-pong)
  Buf<double> part;
  int64_t loaded_rows = 0;  // rows of the input last cast into act[0]
  // standardisation of inputs and targets (set by mlp_fit_scaling /
  // mlp_set_scaling): the network works on (x - x_mu)/x_sd and predicts
  // (y - y_mu)/y_sd
  bool scaled = false;
  Buf<float> xmu, xsd, xisd, ymu, ysd, yisd;
  ~gp_mlp() {
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

thread_local std::string g_mlp_init_error;

void ensure_rows(gp_mlp* m, int64_t rows) {
  if (rows <= m->cap_rows) return;
  m->act.resize(m->L);
  for (int l = 0; l < m->L; ++l) m->act[l].alloc((size_t)rows * (l == 0 ? m->n_pad : m->dims[l]));
  const int nout = m->dims.back();
  m->out.alloc((size_t)rows * nout);
  m->dy.alloc((size_t)rows * nout);
  int wmax = 0;
  for (int d : m->dims) wmax = std::max(wmax, d);
  m->gf.alloc((size_t)rows * wmax);
  m->gb0.alloc((size_t)rows * wmax);
  m->gb1.alloc((size_t)rows * wmax);
  m->part.alloc((size_t)nblk(rows * (int64_t)nout) + 1);
  m->cap_rows = rows;
}

// refresh the transposed BF16 weights from the FP32 masters
void refresh_wt(gp_mlp* m) {
  for (int l = 0; l < m->L; ++l) {
    const int K = m->dims[l], N = m->dims[l + 1], ldt = l == 0 ? m->n_pad : K;
    hipLaunchKernelGGL(k_transpose_bf16, dim3(nblk((int64_t)N * ldt)), dim3(256), 0, m->stream, m->w.p + m->woff[l],
                       m->wbt.p + m->wtoff[l], K, N, ldt);
  }
  MCHK(hipGetLastError());
}

// forward over `rows` rows whose BF16 input is already in act[0]
void forward(gp_mlp* m, int64_t rows) {
  hipStream_t st = m->stream;
  for (int l = 0; l < m->L; ++l) {
    const int N = m->dims[l + 1];
    const int K = l == 0 ? m->n_pad : m->dims[l];  // layer 0: the zero-padded input
    const __bf16* Wt = m->wbt.p + m->wtoff[l];
    const float* b = m->w.p + m->boff[l];
    if (l + 1 < m->L)
      launch_gemm(false, true, m->act[l].p, K, K, Wt, K, K, nullptr, m->act[l + 1].p, b, (int)rows, N, K,
                  EPI_BIAS_RELU, 0, st);
    else
      launch_gemm(false, true, m->act[l].p, K, K, Wt, K, K, m->out.p, nullptr, b, (int)rows, N, K, EPI_BIAS, 0, st);
  }
}

void load_input(gp_mlp* m, const float* X, int64_t rows, int on_device) {
  const int64_t n = rows * m->dims[0];
  Buf<float> tmp;
  const float* src = X;
  if (!on_device) {
    tmp.alloc(n);
    MCHK(hipMemcpyAsync(tmp.p, X, n * sizeof(float), hipMemcpyHostToDevice, m->stream));
    src = tmp.p;
  }
  hipLaunchKernelGGL(k_cast_input, dim3(nblk(rows * m->n_pad)), dim3(256), 0, m->stream, src, m->act[0].p, rows,
                     m->dims[0], m->n_pad, m->scaled ? m->xmu.p : nullptr, m->scaled ? m->xisd.p : nullptr);
  MCHK(hipGetLastError());
  if (!on_device) MCHK(hipStreamSynchronize(m->stream));
  m->loaded_rows = rows;
}

// mean squared error over rows x n_out and the parameter gradient in m->g
double loss_backward(gp_mlp* m, const float* Tgt, int64_t rows, int on_device) {
  hipStream_t st = m->stream;
  const int nout = m->dims.back();
  const int64_t n = rows * nout;
  Buf<float> tmp;
  const float* t = Tgt;
  if (!on_device) {
    tmp.alloc(n);
    MCHK(hipMemcpyAsync(tmp.p, Tgt, n * sizeof(float), hipMemcpyHostToDevice, st));
    t = tmp.p;
  }
  const int nb = nblk(n);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, st, m->out.p, t, m->dy.p, m->gb0.p, m->part.p, n,
                     1.0 / (double)n, nout, m->scaled ? m->ymu.p : nullptr, m->scaled ? m->yisd.p : nullptr);
  MCHK(hipGetLastError());
  // layer L-1 .. 0
  float* gcur_f = m->dy.p;
  __bf16* gcur_b = m->gb0.p;
  __bf16* gnext_b = m->gb1.p;
  for (int l = m->L - 1; l >= 0; --l) {
    const int K = m->dims[l], N = m->dims[l + 1];
    const int lda = l == 0 ? m->n_pad : K;
    // dW_l = act_l^T g  [K x N] (a sum over the rows)
    launch_gemm(true, false, m->act[l].p, lda, (int)rows, gcur_b, N, (int)rows, m->g.p + m->woff[l], nullptr,
                nullptr, K, N, (int)rows, EPI_NONE, 0, st);
    hipLaunchKernelGGL(k_colsum, dim3(nblk(N)), dim3(256), 0, st, gcur_f, m->g.p + m->boff[l], (int)rows, N);
    MCHK(hipGetLastError());
    if (l > 0) {
      // g_prev = g W_l^T, then through the ReLU of layer l-1's output (act_l)
      launch_gemm(false, true, gcur_b, N, N, m->wb.p + m->woff[l], N, N, m->gf.p, nullptr, nullptr, (int)rows, K, N,
                  EPI_NONE, 0, st);
      const int64_t nk = rows * K;
      hipLaunchKernelGGL(k_relu_bwd, dim3(nblk(nk)), dim3(256), 0, st, m->gf.p, m->act[l].p, gnext_b, nk);
      MCHK(hipGetLastError());
      gcur_f = m->gf.p;
      std::swap(gcur_b, gnext_b);
    }
  }
  std::vector<double> hp(nb);
  MCHK(hipMemcpyAsync(hp.data(), m->part.p, nb * sizeof(double), hipMemcpyDeviceToHost, st));
  MCHK(hipStreamSynchronize(st));
  double s = 0.0;
  for (double v : hp) s += v;
  return s / (double)n;
}

void check_dims(const gp_mlp* m, int64_t rows) {
  if (rows < 1 || rows > (int64_t)1 << 30) mfail(GP_EINVAL, "rows must be in [1, 2^30]");
  (void)m;
}

int mguard(gp_mlp* m, const std::function<int()>& f) {
  try {
    const int rc = f();
    if (m) m->err.clear();
    return rc;
  } catch (const MlpError& e) {
    if (m) m->err = e.msg;
    return e.code;
  }
}
}  // namespace

namespace {
void alloc_scaling(gp_mlp* m) {
  const int ni = m->dims[0], no = m->dims.back();
  m->xmu.alloc(ni);
  m->xsd.alloc(ni);
  m->xisd.alloc(ni);
  m->ymu.alloc(no);
  m->ysd.alloc(no);
  m->yisd.alloc(no);
}

void colstats(gp_mlp* m, const float* X, int64_t rows, int ncol, float* mu, float* sd, float* isd) {
  // rows per chunk: at least 2048, and few enough chunks for the grid
  const int64_t chunk = std::max<int64_t>(2048, (rows + 65534) / 65535);
  const int nchunk = (int)((rows + chunk - 1) / chunk);
  Buf<double> part;
  part.alloc((size_t)2 * nchunk * ncol);
  hipLaunchKernelGGL(k_colstats_part, dim3(nblk(ncol), nchunk), dim3(256), 0, m->stream, X, rows, ncol, chunk,
                     part.p);
  hipLaunchKernelGGL(k_colstats_final, dim3(nblk(ncol)), dim3(256), 0, m->stream, part.p, nchunk, ncol, rows, mu,
                     sd, isd);
  MCHK(hipGetLastError());
  MCHK(hipStreamSynchronize(m->stream));
}
}  // namespace

extern "C" {

int mlp_init(gp_mlp** out, int32_t n_in, int32_t width, int32_t hidden_layers, int32_t n_out, uint64_t seed,
             void* hip_stream) {
  if (!out) return GP_EINVAL;
  *out = nullptr;
  gp_mlp* m = nullptr;
  try {
    if (n_in < 1 || width < 1 || hidden_layers < 0 || n_out < 1 || n_in > 65536 || width > 65536 || n_out > 65536)
      mfail(GP_EINVAL, "bad layer sizes");
    m = new gp_mlp();
    if (hip_stream) {
      m->stream = (hipStream_t)hip_stream;
    } else {
      MCHK(hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking));
      m->own_stream = true;
    }
    (void)scratch_address();  // the allocation-free forward's buffer on this device
    m->dims.push_back(n_in);
    for (int l = 0; l < hidden_layers; ++l) m->dims.push_back(width);
    m->dims.push_back(n_out);
    m->L = (int)m->dims.size() - 1;
    m->n_pad = (n_in + 31) / 32 * 32;  // measured 2 % faster than a multiple of 8
    int64_t o = 0;
    for (int l = 0; l < m->L; ++l) {
      m->woff.push_back(o);
      o += (int64_t)m->dims[l] * m->dims[l + 1];
    }
    for (int l = 0; l < m->L; ++l) {
      m->boff.push_back(o);
      o += m->dims[l + 1];
    }
    m->nparam = o;
    // He-uniform weights, zero biases (seeded, host side)
    std::vector<float> w(o, 0.f);
    std::mt19937_64 rng(seed);
    for (int l = 0; l < m->L; ++l) {
      const float a = std::sqrt(6.0f / (float)m->dims[l]);
      std::uniform_real_distribution<float> U(-a, a);
      for (int64_t i = 0; i < (int64_t)m->dims[l] * m->dims[l + 1]; ++i) w[m->woff[l] + i] = U(rng);
    }
    m->w.alloc(o);
    m->g.alloc(o);
    m->m.alloc(o);
    m->v.alloc(o);
    m->wb.alloc(o);
    int64_t ot = 0;
    for (int l = 0; l < m->L; ++l) {
      m->wtoff.push_back(ot);
      ot += (int64_t)m->dims[l + 1] * (l == 0 ? m->n_pad : m->dims[l]);
    }
    m->wbt.alloc(ot);
    MCHK(hipMemcpyAsync(m->w.p, w.data(), o * sizeof(float), hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemsetAsync(m->m.p, 0, o * sizeof(float), m->stream));
    MCHK(hipMemsetAsync(m->v.p, 0, o * sizeof(float), m->stream));
    MCHK(hipMemsetAsync(m->g.p, 0, o * sizeof(float), m->stream));
    hipLaunchKernelGGL(k_cast_bf16, dim3(nblk(o)), dim3(256), 0, m->stream, m->w.p, m->wb.p, o);
    refresh_wt(m);
    MCHK(hipGetLastError());
    MCHK(hipStreamSynchronize(m->stream));
  } catch (const MlpError& e) {
    g_mlp_init_error = e.msg;
    delete m;
    return e.code;
  }
  *out = m;
  return GP_OK;
}

int mlp_num_params(const gp_mlp* m, int64_t* n) {
  if (!m || !n) return GP_EINVAL;
  *n = m->nparam;
  return GP_OK;
}

int mlp_get_params(gp_mlp* m, float* w_out) {
  if (!m) return GP_EINVAL;
  return mguard(m, [&] {
    if (!w_out) mfail(GP_EINVAL, "w_out is NULL");
    MCHK(hipMemcpyAsync(w_out, m->w.p, m->nparam * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return GP_OK;
  });
}

int mlp_set_params(gp_mlp* m, const float* w_in) {
  if (!m) return GP_EINVAL;
  return mguard(m, [&] {
    if (!w_in) mfail(GP_EINVAL, "w_in is NULL");
    for (int64_t i = 0; i < m->nparam; ++i)
      if (!std::isfinite(w_in[i])) mfail(GP_EINVAL, "parameter %lld is not finite", (long long)i);
    MCHK(hipMemcpyAsync(m->w.p, w_in, m->nparam * sizeof(float), hipMemcpyHostToDevice, m->stream));
    hipLaunchKernelGGL(k_cast_bf16, dim3(nblk(m->nparam)), dim3(256), 0, m->stream, m->w.p, m->wb.p, m->nparam);
    refresh_wt(m);
    MCHK(hipGetLastError());
    MCHK(hipStreamSynchronize(m->stream));
    return GP_OK;
  });
}

int mlp_forward(gp_mlp* m, const float* X, int64_t rows, int32_t on_device, float* Y) {
  if (!m) return GP_EINVAL;
  return mguard(m, [&] {
    if (!X || !Y) mfail(GP_EINVAL, "X and Y must not be NULL");
    check_dims(m, rows);
    ensure_rows(m, rows);
    load_input(m, X, rows, on_device);
    forward(m, rows);
    const int64_t n = rows * m->dims.back();
    const float* src = m->out.p;
    if (m->scaled) {  // back to target units, in place in the dY buffer
      hipLaunchKernelGGL(k_unscale, dim3(nblk(n)), dim3(256), 0, m->stream, m->out.p, m->dy.p, n, m->dims.back(),
                         m->ymu.p, m->ysd.p);
      MCHK(hipGetLastError());
      src = m->dy.p;
    }
    MCHK(hipMemcpyAsync(Y, src, n * sizeof(float), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    return GP_OK;
  });
}

int mlp_forward_noalloc(gp_mlp* m, const float* X_dev, int64_t rows, float* Y_dev, int64_t* max_rows) {
  if (!m) return GP_EINVAL;
  return mguard(m, [&] {
    // two BF16 buffers of rows x (widest layer input) elements
    int wmax = m->n_pad;
    for (int l = 1; l < m->L; ++l) wmax = std::max(wmax, m->dims[l]);
    const int64_t per_row = 2 * (int64_t)wmax * (int64_t)sizeof(__bf16);
    const int64_t cap = (int64_t)(kScratchBytes / (size_t)per_row);
    if (max_rows) *max_rows = cap;
    if (!X_dev || !Y_dev) mfail(GP_EINVAL, "X and Y must not be NULL");
    check_dims(m, rows);
    if (rows > cap)
      mfail(GP_EINVAL, "%lld rows exceed the %lld that the %zu-byte forward scratch holds for this network",
            (long long)rows, (long long)cap, kScratchBytes);
    unsigned char* base = (unsigned char*)scratch_address();
    __bf16* buf[2] = {(__bf16*)base, (__bf16*)(base + (size_t)rows * wmax * sizeof(__bf16))};
    hipStream_t st = m->stream;
    // input cast (and standardisation) into the zero-padded layout; every
    // entry of [rows x n_pad] is written, so nothing needs clearing
    hipLaunchKernelGGL(k_cast_input, dim3(nblk(rows * m->n_pad)), dim3(256), 0, st, X_dev, buf[0], rows,
                       m->dims[0], m->n_pad, m->scaled ? m->xmu.p : nullptr, m->scaled ? m->xisd.p : nullptr);
    MCHK(hipGetLastError());
    for (int l = 0; l < m->L; ++l) {
      const int N = m->dims[l + 1];
      const int K = l == 0 ? m->n_pad : m->dims[l];
      const __bf16* Wt = m->wbt.p + m->wtoff[l];
      const float* b = m->w.p + m->boff[l];
      if (l + 1 < m->L)
        launch_gemm(false, true, buf[l & 1], K, K, Wt, K, K, nullptr, buf[(l + 1) & 1], b, (int)rows, N, K,
                    EPI_BIAS_RELU, 0, st);
      else
        launch_gemm(false, true, buf[l & 1], K, K, Wt, K, K, Y_dev, nullptr, b, (int)rows, N, K, EPI_BIAS, 0, st);
    }
    if (m->scaled) {  // back to target units, in place
      const int64_t n = rows * m->dims.back();
      hipLaunchKernelGGL(k_unscale, dim3(nblk(n)), dim3(256), 0, st, Y_dev, Y_dev, n, m->dims.back(), m->ymu.p,
                         m->ysd.p);
      MCHK(hipGetLastError());
    }
    return GP_OK;
  });
}

int mlp_loss_grad(gp_mlp* m, const float* X, const float* T, int64_t rows, int32_t on_device, double* loss,
                  float* grad_out) {
  if (!m) return GP_EINVAL;
  return mguard(m, [&] {
    if (!X || !T) mfail(GP_EINVAL, "X and T must not be NULL");
    check_dims(m, rows);
    ensure_rows(m, rows);
    load_input(m, X, rows, on_device);
    forward(m, rows);
    const double l = loss_backward(m, T, rows, on_device);
    if (loss) *loss = l;
    if (grad_out) {
      MCHK(hipMemcpyAsync(grad_out, m->g.p, m->nparam * sizeof(float), hipMemcpyDeviceToHost, m->stream));
      MCHK(hipStreamSynchronize(m->stream));
    }
    return GP_OK;
  });
}

int mlp_adam_step(gp_mlp* m, const float* X, const float* T, int64_t rows, int32_t on_device, double lr,
                  double* loss) {
  if (!m) return GP_EINVAL;
  return mguard(m, [&] {
    if (!X || !T) mfail(GP_EINVAL, "X and T must not be NULL");
    if (!(lr > 0) || !std::isfinite(lr)) mfail(GP_EINVAL, "lr must be > 0");
    check_dims(m, rows);
    ensure_rows(m, rows);
    load_input(m, X, rows, on_device);
    forward(m, rows);
    const double l = loss_backward(m, T, rows, on_device);
    if (loss) *loss = l;
    m->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
    // weights (with their BF16 copies) then biases
    const int64_t nw = m->boff[0];
    hipLaunchKernelGGL(k_adam, dim3(nblk(nw)), dim3(256), 0, m->stream, m->w.p, m->g.p, m->m.p, m->v.p, m->wb.p, nw,
                       (float)lr, b1, b2, 1e-8f, c1, c2);
    const int64_t nbias = m->nparam - nw;
    hipLaunchKernelGGL(k_adam, dim3(nblk(nbias)), dim3(256), 0, m->stream, m->w.p + nw, m->g.p + nw, m->m.p + nw,
                       m->v.p + nw, (__bf16*)nullptr, nbias, (float)lr, b1, b2, 1e-8f, c1, c2);
    MCHK(hipGetLastError());
    refresh_wt(m);
    MCHK(hipStreamSynchronize(m->stream));
    return GP_OK;
  });
}


int mlp_fit_scaling(gp_mlp* m, const float* X, const float* T, int64_t rows, int32_t on_device) {
  if (!m) return GP_EINVAL;
  return mguard(m, [&] {
    if (!X || !T) mfail(GP_EINVAL, "X and T must not be NULL");
    check_dims(m, rows);
    const int ni = m->dims[0], no = m->dims.back();
    Buf<float> hx, ht;
    const float *x = X, *t = T;
    if (!on_device) {
      hx.alloc((size_t)rows * ni);
      ht.alloc((size_t)rows * no);
      MCHK(hipMemcpyAsync(hx.p, X, (size_t)rows * ni * sizeof(float), hipMemcpyHostToDevice, m->stream));
      MCHK(hipMemcpyAsync(ht.p, T, (size_t)rows * no * sizeof(float), hipMemcpyHostToDevice, m->stream));
      x = hx.p;
      t = ht.p;
    }
    alloc_scaling(m);
    colstats(m, x, rows, ni, m->xmu.p, m->xsd.p, m->xisd.p);
    colstats(m, t, rows, no, m->ymu.p, m->ysd.p, m->yisd.p);
    m->scaled = true;
    return GP_OK;
  });
}

int mlp_get_scaling(gp_mlp* m, float* x_mu, float* x_sd, float* y_mu, float* y_sd) {
  if (!m) return GP_EINVAL;
  return mguard(m, [&] {
    if (!m->scaled) mfail(GP_ESTATE, "no scaling set");
    const int ni = m->dims[0], no = m->dims.back();
    auto get = [&](float* dst, const Buf<float>& b, int n) {
      if (dst) MCHK(hipMemcpyAsync(dst, b.p, n * sizeof(float), hipMemcpyDeviceToHost, m->stream));
    };
    get(x_mu, m->xmu, ni);
    get(x_sd, m->xsd, ni);
    get(y_mu, m->ymu, no);
    get(y_sd, m->ysd, no);
    MCHK(hipStreamSynchronize(m->stream));
    return GP_OK;
  });
}

int mlp_set_scaling(gp_mlp* m, const float* x_mu, const float* x_sd, const float* y_mu, const float* y_sd) {
  if (!m) return GP_EINVAL;
  return mguard(m, [&] {
    if (!x_mu || !x_sd || !y_mu || !y_sd) mfail(GP_EINVAL, "scaling arrays must not be NULL");
    const int ni = m->dims[0], no = m->dims.back();
    std::vector<float> xi(ni), yi(no);
    for (int c = 0; c < ni; ++c) {
      if (!std::isfinite(x_mu[c]) || !(x_sd[c] > 0.f) || !std::isfinite(x_sd[c])) mfail(GP_EINVAL, "bad input scaling");
      xi[c] = 1.f / x_sd[c];
    }
    for (int c = 0; c < no; ++c) {
      if (!std::isfinite(y_mu[c]) || !(y_sd[c] > 0.f) || !std::isfinite(y_sd[c])) mfail(GP_EINVAL, "bad target scaling");
      yi[c] = 1.f / y_sd[c];
    }
    alloc_scaling(m);
    MCHK(hipMemcpyAsync(m->xmu.p, x_mu, ni * sizeof(float), hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemcpyAsync(m->xsd.p, x_sd, ni * sizeof(float), hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemcpyAsync(m->xisd.p, xi.data(), ni * sizeof(float), hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemcpyAsync(m->ymu.p, y_mu, no * sizeof(float), hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemcpyAsync(m->ysd.p, y_sd, no * sizeof(float), hipMemcpyHostToDevice, m->stream));
    MCHK(hipMemcpyAsync(m->yisd.p, yi.data(), no * sizeof(float), hipMemcpyHostToDevice, m->stream));
    MCHK(hipStreamSynchronize(m->stream));
    m->scaled = true;
    return GP_OK;
  });
}

int mlp_time_forward(gp_mlp* m, int64_t rows, int32_t iters, double* ms_out) {
  if (!m) return GP_EINVAL;
  return mguard(m, [&] {
    if (!ms_out || iters < 1) mfail(GP_EINVAL, "ms_out must not be NULL and iters >= 1");
    if (rows < 1 || rows > m->loaded_rows) mfail(GP_ESTATE, "time only rows already loaded by a forward call");
    hipEvent_t e0, e1;
    MCHK(hipEventCreate(&e0));
    MCHK(hipEventCreate(&e1));
    forward(m, rows);  // untimed
    MCHK(hipEventRecord(e0, m->stream));
    for (int i = 0; i < iters; ++i) forward(m, rows);
    MCHK(hipEventRecord(e1, m->stream));
    MCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    MCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = ms / iters;
    return GP_OK;
  });
}

// plain GEMM through the same kernel (for tests): C = op(A) op(B), BF16 in
// (host FP32 rounded to BF16), FP32 out.  Host pointers.
int mlp_gemm_test(const float* A, const float* B, float* C, int32_t M, int32_t N, int32_t K, int32_t ta,
                  int32_t tb) {
  try {
    if (!A || !B || !C || M < 1 || N < 1 || K < 1) return GP_EINVAL;
    hipStream_t st = nullptr;
    Buf<float> fa, fb, fc;
    Buf<__bf16> ba, bb;
    const int64_t na = (int64_t)M * K, nb = (int64_t)K * N, nc = (int64_t)M * N;
    fa.alloc(na);
    fb.alloc(nb);
    fc.alloc(nc);
    ba.alloc(na);
    bb.alloc(nb);
    MCHK(hipMemcpy(fa.p, A, na * sizeof(float), hipMemcpyHostToDevice));
    MCHK(hipMemcpy(fb.p, B, nb * sizeof(float), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_cast_bf16, dim3(nblk(na)), dim3(256), 0, st, fa.p, ba.p, na);
    hipLaunchKernelGGL(k_cast_bf16, dim3(nblk(nb)), dim3(256), 0, st, fb.p, bb.p, nb);
    launch_gemm(ta != 0, tb != 0, ba.p, ta ? M : K, K, bb.p, tb ? K : N, K, fc.p, nullptr, nullptr, M, N, K,
                EPI_NONE, 0, st);
    MCHK(hipMemcpy(C, fc.p, nc * sizeof(float), hipMemcpyDeviceToHost));
    return GP_OK;
  } catch (const MlpError& e) {
    g_mlp_init_error = e.msg;
    return e.code;
  }
}

void mlp_free(gp_mlp* m) {
  if (!m) return;
  if (m->stream) (void)hipStreamSynchronize(m->stream);
  delete m;
}

const char* mlp_last_error(const gp_mlp* m) { return m ? m->err.c_str() : g_mlp_init_error.c_str(); }

}  // extern "C"
