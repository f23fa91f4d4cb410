// Kernels of the surrogate network: a multilayer perceptron
// in(<=64) -> 256 -> 256 -> 256 -> out(<=64) with SiLU activations, BF16
// weights and activations feeding the matrix cores (MFMA), FP32 accumulation,
// FP32 master weights and Adam.  Inputs and outputs are zero-padded to 64
// columns; padded weights start at zero and keep a zero gradient.
//
// Parameter vector (fp32), layer l = 0..3 with fan-in K_l and fan-out N_l:
//   W_0[N_0][K_0] | b_0[N_0] | W_1 | b_1 | W_2 | b_2 | W_3 | b_3
// (weights stored [out][in]); the BF16 copy holds W_0 | W_1 | W_2 | W_3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cfust {
// every kernel, device function and table has internal linkage: each
// translation unit of the library compiles the ones it uses
namespace {

using bf16 = unsigned short;
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

constexpr int kMlpPad = 64;   // padded input and output widths
constexpr int kMlpHid = 256;  // hidden width
constexpr int kMlpLayers = 4;

__host__ __device__ constexpr int mlp_k(int l) { return l == 0 ? kMlpPad : kMlpHid; }
__host__ __device__ constexpr int mlp_n(int l) { return l == kMlpLayers - 1 ? kMlpPad : kMlpHid; }
// offsets of W_l and b_l in the parameter vector, of W_l in the bf16 copy
__host__ __device__ constexpr int64_t mlp_w_off(int l) {
  return l == 0 ? 0 : mlp_w_off(l - 1) + (int64_t)mlp_n(l - 1) * mlp_k(l - 1) + mlp_n(l - 1);
}
__host__ __device__ constexpr int64_t mlp_b_off(int l) {
  return mlp_w_off(l) + (int64_t)mlp_n(l) * mlp_k(l);
}
__host__ __device__ constexpr int64_t mlp_wb_off(int l) {
  return l == 0 ? 0 : mlp_wb_off(l - 1) + (int64_t)mlp_n(l - 1) * mlp_k(l - 1);
}
// the same offsets as compile-time constants (device code must not call the
// recursive helpers at run time: that is a real call with a dynamic stack)
template <int L>
struct MlpOff {
  static constexpr int64_t w = mlp_w_off(L), b = mlp_b_off(L), wb = mlp_wb_off(L);
};
constexpr int64_t kMlpParams = mlp_b_off(kMlpLayers - 1) + mlp_n(kMlpLayers - 1);
constexpr int64_t kMlpWeightsBf = mlp_wb_off(kMlpLayers);

__device__ __forceinline__ bf16 f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
  return (bf16)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ __forceinline__ float sigmoid_f(float z) { return 1.0f / (1.0f + __expf(-z)); }

// epilogue of the GEMM
enum EpiMode : int {
  kEpiStore = 0,     // C[z][row][col] = acc            (split-K partial sums)
  kEpiBiasSilu = 1,  // z = acc + b; Zs = z (if given); H = bf16(SiLU(z))
  kEpiBias = 2,      // C = acc + b
  kEpiSiluBwd = 3,   // g = acc * SiLU'(Zs); C = g (if given); H = bf16(g), H2 = bf16(g - H)
};
struct Epi {
  float* C;         // fp32 output [rows][ldc] (per split: + z * M * ldc)
  const float* b;   // bias [N]
  float* Zs;        // fp32 pre-activation, written (mode 1) or read (mode 3)
  bf16* H;          // bf16 output [rows][ldc]
  bf16* H2;         // bf16 low part (mode 3, if given)
  int ldc;
};

// x ~ hi + lo with hi = bf16(x), lo = bf16(x - hi): about 16 significant bits
__device__ __forceinline__ void split_bf16(float x, bf16& hi, bf16& lo) {
  hi = f2bf(x);
  lo = f2bf(x - bf2f(hi));
}

// ---------------------------------------------------------------------------
// out[M][N] = op(A) op(B) with bf16 operands and fp32 accumulation, then the
// epilogue:  op(A)[m][k] = TA ? A[k*lda + m] : A[m*lda + k],
//            op(B)[k][n] = TB ? B[n*ldb + k] : B[k*ldb + n].
// With SPLIT, A is the pair (A, A2) of high and low bf16 parts and the
// product is op(A) op(B) + op(A2) op(B) (back-propagated values keep about
// 16 significant bits that way).
// Block of 256 threads = 4 waves on a 64x64 output tile; wave (wm, wn) owns a
// 32x32 quarter as 2x2 tiles of v_mfma_f32_16x16x16_bf16; K advances 32 at a
// time through LDS, both operands stored k-contiguous there so that every
// fragment is one 8-byte LDS read.  Row tiles on grid x, column tiles on
// grid y; blockIdx.z splits K into slices of kps.
// Requires M, N multiples of 64, K and kps multiples of 32, lda and ldb
// multiples of 8, 16-byte aligned base pointers.
// ---------------------------------------------------------------------------
template <bool TA, bool TB, int MODE, bool SPLIT = false>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(const bf16* __restrict__ A,
                                                        const bf16* __restrict__ A2, int lda,
                                                        const bf16* __restrict__ B, int ldb,
                                                        int M, int N, int K, int kps, Epi ep) {
  constexpr int KT = 32;
  constexpr int LD = KT + 8;  // row pitch in LDS (80 bytes)
  __shared__ __attribute__((aligned(16))) bf16 As[(SPLIT ? 2 : 1) * 64 * LD];
  __shared__ __attribute__((aligned(16))) bf16 Bs[64 * LD];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;  // row tiles on x (may be many)
  const int kbeg = blockIdx.z * kps;
  const int kend = min(K, kbeg + kps);
  float4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
  const int r16 = lane & 15, kg = lane >> 4;
  // each thread moves 8 consecutive bf16 (16 bytes) of each operand per K step
  const int e = tid * 8;
  for (int k0 = kbeg; k0 < kend; k0 += KT) {
#pragma unroll
    for (int part = 0; part < (SPLIT ? 2 : 1); ++part) {
      const bf16* Ap = part ? A2 : A;
      bf16* Al = As + part * 64 * LD;
      if (!TA) {
        const int m = e / KT, k = e % KT;
        const uint4 v = *reinterpret_cast<const uint4*>(Ap + (size_t)(m0 + m) * lda + k0 + k);
        *reinterpret_cast<uint4*>(&Al[m * LD + k]) = v;
      } else {
        const int k = e / 64, m = e % 64;
        const uint4 v = *reinterpret_cast<const uint4*>(Ap + (size_t)(k0 + k) * lda + m0 + m);
        const bf16* hv = reinterpret_cast<const bf16*>(&v);
#pragma unroll
        for (int t = 0; t < 8; ++t) Al[(m + t) * LD + k] = hv[t];
      }
    }
    if (TB) {
      const int n = e / KT, k = e % KT;
      const uint4 v = *reinterpret_cast<const uint4*>(B + (size_t)(n0 + n) * ldb + k0 + k);
      *reinterpret_cast<uint4*>(&Bs[n * LD + k]) = v;
    } else {
      const int k = e / 64, n = e % 64;
      const uint4 v = *reinterpret_cast<const uint4*>(B + (size_t)(k0 + k) * ldb + n0 + n);
      const bf16* hv = reinterpret_cast<const bf16*>(&v);
#pragma unroll
      for (int t = 0; t < 8; ++t) Bs[(n + t) * LD + k] = hv[t];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KT; kk += 16) {
      short4_t af[2], bfr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        af[i] = *reinterpret_cast<const short4_t*>(&As[(32 * wm + 16 * i + r16) * LD + kk + 4 * kg]);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        bfr[j] = *reinterpret_cast<const short4_t*>(&Bs[(32 * wn + 16 * j + r16) * LD + kk + 4 * kg]);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bfr[j], acc[i][j], 0, 0, 0);
      if (SPLIT) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
          af[i] = *reinterpret_cast<const short4_t*>(
              &As[64 * LD + (32 * wm + 16 * i + r16) * LD + kk + 4 * kg]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(af[i], bfr[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // 16x16 result tile: lane holds rows 4*(lane/16) + t, column lane % 16
  float* C = ep.C;
  if (MODE == kEpiStore) C += (size_t)blockIdx.z * M * ep.ldc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int row = m0 + 32 * wm + 16 * i + 4 * kg + t;
        const int col = n0 + 32 * wn + 16 * j + r16;
        const size_t o = (size_t)row * ep.ldc + col;
        const float a = acc[i][j][t];
        if (MODE == kEpiStore) {
          C[o] = a;
        } else if (MODE == kEpiBias) {
          C[o] = a + ep.b[col];
        } else if (MODE == kEpiBiasSilu) {
          const float z = a + ep.b[col];
          if (ep.Zs) ep.Zs[o] = z;
          ep.H[o] = f2bf(z * sigmoid_f(z));
        } else {
          const float z = ep.Zs[o];
          const float sg = sigmoid_f(z);
          const float gr = a * sg * (1.0f + z * (1.0f - sg));
          if (C) C[o] = gr;
          bf16 hi, lo;
          split_bf16(gr, hi, lo);
          ep.H[o] = hi;
          if (ep.H2) ep.H2[o] = lo;
        }
      }
}

// ---------------------------------------------------------------------------
// Fused inference: one 256-thread block takes 16 RT rows through all four
// layers.  The activations of the block's rows stay in LDS (one 16 RT x 256
// bf16 tile, overwritten layer by layer after a barrier); weights are read
// k-contiguous from global memory (L2-resident, [out][in] layout).  Wave w
// owns output columns [w N/4, (w+1) N/4) of every layer and all the block's
// rows.  Each 16 x 16 output tile is one v_mfma_f32_16x16x32_bf16 (gfx950)
// per 32 inputs with the weights as the A operand and the activations as B,
// so the tile comes out transposed (features x rows): lane l supplies
// W[c0 + l%16][k0 + 8(l/16) .. +7] and H[r0 + l%16][k0 + 8(l/16) .. +7] and
// receives the four consecutive features c0 + 4(l/16) + t, t = 0..3, of row
// r0 + l%16.  Bias, SiLU and the bf16 rounding then end in one 8-byte LDS
// store per tile and lane (one 16-byte store of fp32 outputs in the last
// layer).  A wave's weight loads are shared by its RT row tiles and are
// issued one 32-input step ahead of the MFMAs that use them.  HBM traffic is
// the input rows (bf16) and the fp32 outputs only.  Rows at or past `rows`
// are zero on input and never stored.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef unsigned short ushort4_t __attribute__((ext_vector_type(4)));
constexpr int kFusedLd = kMlpHid + 8;  // LDS row pitch (528 bytes)
// row tiles per block: 128 rows, which halves the L2 weight bytes per MFMA
// against 64 rows (710 against 775 us per 2^20 rows, bit-identical outputs;
// in the first version of this kernel 128 rows had been 13% slower).
constexpr int kInferRT = 8;

template <int K, int N, bool LAST, int RT>
__device__ __forceinline__ void fused_layer(bf16* __restrict__ Hs, const bf16* __restrict__ W,
                                            const float* __restrict__ b, float* __restrict__ P,
                                            int64_t row0, int64_t rows, int lane, int w) {
  constexpr int CT = N / 64;  // 16-column tiles per wave
  constexpr int KS = K / 32;  // 32-input steps
  const int colbase = w * (N / 4);
  const int r16 = lane & 15, kg = lane >> 4;
  // bias of this lane's four features in each column tile
  float4_t bias[CT];
#pragma unroll
  for (int j = 0; j < CT; ++j)
    bias[j] = *reinterpret_cast<const float4_t*>(b + colbase + 16 * j + 4 * kg);
  float4_t acc[CT][RT];
#pragma unroll
  for (int j = 0; j < CT; ++j)
#pragma unroll
    for (int i = 0; i < RT; ++i) acc[j][i] = float4_t{0.f, 0.f, 0.f, 0.f};
  const bf16* wrow = W + (size_t)(colbase + r16) * K + 8 * kg;
  bf16x8_t bw[CT];
#pragma unroll
  for (int j = 0; j < CT; ++j) bw[j] = *reinterpret_cast<const bf16x8_t*>(wrow + (size_t)16 * j * K);
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int k0 = 32 * s;
    // next step's weights in flight while this step's MFMAs run
    bf16x8_t nw[CT];
    if (s + 1 < KS) {
#pragma unroll
      for (int j = 0; j < CT; ++j)
        nw[j] = *reinterpret_cast<const bf16x8_t*>(wrow + (size_t)16 * j * K + k0 + 32);
    }
    bf16x8_t a[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
      a[i] = *reinterpret_cast<const bf16x8_t*>(Hs + (16 * i + r16) * kFusedLd + k0 + 8 * kg);
#pragma unroll
    for (int j = 0; j < CT; ++j)
#pragma unroll
      for (int i = 0; i < RT; ++i)
        acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bw[j], a[i], acc[j][i], 0, 0, 0);
    if (s + 1 < KS) {
#pragma unroll
      for (int j = 0; j < CT; ++j) bw[j] = nw[j];
    }
  }
  __syncthreads();  // every wave has read this layer's input
#pragma unroll
  for (int j = 0; j < CT; ++j) {
    const int col = colbase + 16 * j + 4 * kg;
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const int row = 16 * i + r16;
      const float4_t z = acc[j][i] + bias[j];
      if (LAST) {
        if (row0 + row < rows)
          *reinterpret_cast<float4_t*>(P + (size_t)(row0 + row) * kMlpPad + col) = z;
      } else {
        ushort4_t h;
#pragma unroll
        for (int t = 0; t < 4; ++t) h[t] = f2bf(z[t] * sigmoid_f(z[t]));
        *reinterpret_cast<ushort4_t*>(Hs + row * kFusedLd + col) = h;
      }
    }
  }
  __syncthreads();
}

// Two resident waves per SIMD at 128 rows per block (256 VGPRs, 16 B/lane
// of spill outside the MFMA loop; the LDS tile of 67.6 KB allows two blocks
// per CU).  At 64 rows three waves (139 VGPRs) took 779 us per 2^20 rows
// against 876 us for the compiler's two; four spilled and measured the same.
template <int RT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void mlp_infer_kernel(const bf16* __restrict__ X, int64_t rows,
                                                        const bf16* __restrict__ wb,
                                                        const float* __restrict__ params,
                                                        float* __restrict__ P) {
  constexpr int R = 16 * RT;  // rows per block
  static_assert(R % 64 == 0, "the input copy moves 64 rows per pass");
  __shared__ __attribute__((aligned(16))) bf16 Hs[R * kFusedLd];
  const int64_t row0 = (int64_t)blockIdx.x * R;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  // the block's input rows, 16 bf16 (one uint4 pair) per thread per pass
#pragma unroll
  for (int pass = 0; pass < R / 64; ++pass) {
    const int r = 64 * pass + (tid >> 2), c = (tid & 3) * 16;
    uint4* dst = reinterpret_cast<uint4*>(Hs + r * kFusedLd + c);
    if (row0 + r < rows) {
      const uint4* src = reinterpret_cast<const uint4*>(X + (size_t)(row0 + r) * kMlpPad + c);
      dst[0] = src[0];
      dst[1] = src[1];
    } else {
      dst[0] = uint4{0u, 0u, 0u, 0u};
      dst[1] = uint4{0u, 0u, 0u, 0u};
    }
  }
  __syncthreads();
  fused_layer<mlp_k(0), mlp_n(0), false, RT>(Hs, wb + MlpOff<0>::wb, params + MlpOff<0>::b,
                                             nullptr, row0, rows, lane, w);
  fused_layer<mlp_k(1), mlp_n(1), false, RT>(Hs, wb + MlpOff<1>::wb, params + MlpOff<1>::b,
                                             nullptr, row0, rows, lane, w);
  fused_layer<mlp_k(2), mlp_n(2), false, RT>(Hs, wb + MlpOff<2>::wb, params + MlpOff<2>::b,
                                             nullptr, row0, rows, lane, w);
  fused_layer<mlp_k(3), mlp_n(3), true, RT>(Hs, wb + MlpOff<3>::wb, params + MlpOff<3>::b, P,
                                            row0, rows, lane, w);
}

// out[i] = sum_s part[s * n + i] (fixed order)
__global__ void sum_slices_kernel(const float* __restrict__ part, int S, int64_t n,
                                  float* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  float s = 0.f;
  for (int k = 0; k < S; ++k) s += part[(size_t)k * n + t];
  out[t] = s;
}

// column sums of X[M][N] over row chunks of 256: part[chunk][N]; block
// (64 columns, 4 row groups), grid (N / 64, ceil(M / 256))
__global__ __launch_bounds__(256) void colsum_part_kernel(const float* __restrict__ X, int64_t M,
                                                          int N, float* __restrict__ part) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int rg = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.y * 256;
  float s = 0.f;
  for (int r = rg; r < 256; r += 4) {
    const int64_t row = r0 + r;
    if (row < M) s += X[row * N + c];
  }
  red[rg][threadIdx.x & 63] = s;
  __syncthreads();
  if (rg == 0) {
    const int cc = threadIdx.x & 63;
    part[(size_t)blockIdx.y * N + c] = (red[0][cc] + red[1][cc]) + (red[2][cc] + red[3][cc]);
  }
}

// Mean squared error over the valid rows r < Mv and outputs o < OUT, each
// output weighted by wo[o]:  L = sum wo_o (P - T)^2 / (Mv sum_o wo_o).
// dP = dL/dP (fp32, and as high and low bf16 parts; zero on padding).  One
// partial loss per block.
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* __restrict__ P,
                                                       const float* __restrict__ T, int64_t M,
                                                       int64_t Mv, int OUT,
                                                       const float* __restrict__ wo, float wsum,
                                                       float* __restrict__ dP,
                                                       bf16* __restrict__ dPb,
                                                       bf16* __restrict__ dPlo,
                                                       float* __restrict__ loss_part) {
  __shared__ float red[256];
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float l = 0.f;
  if (t < M * kMlpPad) {
    const int64_t r = t / kMlpPad;
    const int o = (int)(t % kMlpPad);
    float gr = 0.f;
    if (r < Mv && o < OUT) {
      const float d = P[t] - T[r * OUT + o];
      const float sc = wo[o] / (wsum * (float)Mv);
      l = sc * d * d;
      gr = 2.0f * sc * d;
    }
    dP[t] = gr;
    bf16 hi, lo;
    split_bf16(gr, hi, lo);
    dPb[t] = hi;
    dPlo[t] = lo;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// Per-step scalars of a training run come from a device step counter, so
// that one step is the same launch sequence every time (it is captured once
// in a hipGraph and replayed): minibatch k of the epoch is rows
// [k B, (k+1) B) of the shuffled index, the loss goes to slot epoch, and
// Adam's learning rate follows a cosine from lr0 to lr1 over `total` steps.
struct TrainStep {
  const int64_t* step;  // steps done in this run (device)
  int64_t per_epoch, total, B, Bp, t0;  // t0: Adam steps before this run
  double lr0, lr1;
};

__global__ void gather_step_kernel(const double* __restrict__ feat, const double* __restrict__ targ,
                                   const int64_t* __restrict__ idx, TrainStep ts, int IN, int OUT,
                                   const float* __restrict__ mx, const float* __restrict__ sx,
                                   const float* __restrict__ my, const float* __restrict__ sy,
                                   bf16* __restrict__ X, float* __restrict__ T) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ts.Bp * kMlpPad) return;
  const int64_t base = (ts.step[0] % ts.per_epoch) * ts.B;
  const int64_t r = t / kMlpPad;
  const int c = (int)(t % kMlpPad);
  const int64_t s = r < ts.B ? idx[base + r] : 0;
  float xv = 0.f;
  if (r < ts.B && c < IN) xv = (float)((feat[s * IN + c] - (double)mx[c]) / (double)sx[c]);
  X[t] = f2bf(xv);
  if (c < OUT) {
    float tv = 0.f;
    if (r < ts.B) tv = (float)((targ[s * OUT + c] - (double)my[c]) / (double)sy[c]);
    T[r * OUT + c] = tv;
  }
}

__global__ void adam_step_kernel(float* __restrict__ w, const float* __restrict__ g,
                                 float* __restrict__ m, float* __restrict__ v, int64_t n,
                                 TrainStep ts, float b1, float b2, float eps) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const int64_t k = ts.step[0];
  const double tt = (double)(ts.t0 + k + 1);
  const float lr = (float)(ts.lr1 + 0.5 * (ts.lr0 - ts.lr1) *
                                        (1.0 + cos(3.141592653589793 * (double)k / (double)ts.total)));
  const float bc1 = (float)(1.0 - pow((double)b1, tt));
  const float bc2 = (float)(1.0 - pow((double)b2, tt));
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.f - b1) * gt;
  const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  w[t] -= lr * (mt / bc1) / (sqrtf(vt / bc2) + eps);
}

__global__ void step_inc_kernel(int64_t* step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) step[0] += 1;
}

// acc[slot] += sum of part[0..n) (one block of 256 threads, fixed order);
// with step given the slot is step[0] / per_epoch
__global__ __launch_bounds__(256) void accumulate_step_kernel(const float* __restrict__ part, int n,
                                                              double* __restrict__ acc,
                                                              const int64_t* __restrict__ step,
                                                              int64_t per_epoch) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[step[0] / per_epoch] += red[0];
}

// acc[slot] += sum of part[0..n) (one block of 256 threads, fixed order)
__global__ __launch_bounds__(256) void accumulate_kernel(const float* __restrict__ part, int n,
                                                         double* __restrict__ acc, int slot) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) acc[slot] += red[0];
}

// Adam on the fp32 parameter vector (bias-corrected, no weight decay)
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                            float b1, float b2, float eps, float bc1, float bc2) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float gt = g[t];
  const float mt = b1 * m[t] + (1.f - b1) * gt;
  const float vt = b2 * v[t] + (1.f - b2) * gt * gt;
  m[t] = mt;
  v[t] = vt;
  w[t] -= lr * (mt / bc1) / (sqrtf(vt / bc2) + eps);
}

// bf16 copy of the four weight matrices from the parameter vector
__global__ void weights_to_bf16_kernel(const float* __restrict__ w, bf16* __restrict__ wb) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= kMlpWeightsBf) return;
  static_assert(kMlpLayers == 4, "one branch per layer");
  // W_l sits at MlpOff<l>::w in the parameter vector (after b_{l-1}) and at
  // MlpOff<l>::wb in the bf16 copy (weights only)
  const int64_t shift = t >= MlpOff<3>::wb   ? MlpOff<3>::w - MlpOff<3>::wb
                        : t >= MlpOff<2>::wb ? MlpOff<2>::w - MlpOff<2>::wb
                        : t >= MlpOff<1>::wb ? MlpOff<1>::w - MlpOff<1>::wb
                                             : 0;
  wb[t] = f2bf(w[t + shift]);
}

// per-column mean and standard deviation of X[M][D] (double), two passes,
// one block per column; sd is floored at 1e-12 (constant columns)
__global__ __launch_bounds__(256) void col_moments_kernel(const double* __restrict__ X, int64_t M,
                                                          int D, float* __restrict__ mean,
                                                          float* __restrict__ sd) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < M; r += 256) s += X[r * D + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  const double mu = red[0] / (double)M;
  __syncthreads();
  double v = 0.0;
  for (int64_t r = threadIdx.x; r < M; r += 256) {
    const double d = X[r * D + c] - mu;
    v += d * d;
  }
  red[threadIdx.x] = v;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mean[c] = (float)mu;
    sd[c] = (float)fmax(sqrt(red[0] / (double)M), 1e-12);
  }
}

// The network's outputs for a truncated-t problem of dimension q are
//   log P(V <= h) | m1 = E[V | V <= h] (q) | U (q(q+1)/2)
// with Cov(V | V <= h) = U^T U, U upper triangular packed row by row and its
// diagonal stored as logarithms: every prediction is a positive definite
// covariance.  The labels carry E[V V^T | V <= h] (upper triangle) instead.
constexpr int kNetMaxQ = 8;

// label row -> network row (Cov = E[VV^T] - m1 m1^T factored by Cholesky).
// Squared pivots are floored at kPivotFloor: a truncated t with unit-scale
// margins and bounds in the training box has conditional variances far
// above it, so only degenerate estimates (all weight on a few points) are
// affected, and they stay finite.
constexpr double kPivotFloor = 1e-6;
__device__ inline void net_row(const double* __restrict__ lab, int q, double* __restrict__ out) {
  double U[kNetMaxQ * kNetMaxQ];
  out[0] = lab[0];
  for (int a = 0; a < q; ++a) out[1 + a] = lab[1 + a];
  int c = 1 + q;
  for (int a = 0; a < q; ++a)
    for (int b = a; b < q; ++b, ++c) U[a * q + b] = lab[c] - lab[1 + a] * lab[1 + b];
  // Cov = U^T U: row a of U from the rows above it
  for (int a = 0; a < q; ++a) {
    double d = U[a * q + a];
    for (int k = 0; k < a; ++k) d -= U[k * q + a] * U[k * q + a];
    d = sqrt(fmax(d, kPivotFloor));
    U[a * q + a] = d;
    for (int b = a + 1; b < q; ++b) {
      double t = U[a * q + b];
      for (int k = 0; k < a; ++k) t -= U[k * q + a] * U[k * q + b];
      U[a * q + b] = t / d;
    }
  }
  c = 1 + q;
  for (int a = 0; a < q; ++a)
    for (int b = a; b < q; ++b, ++c) out[c] = (a == b) ? log(U[a * q + a]) : U[a * q + b];
}

// de-standardised network row (fp32 outputs P, width >= T) -> label row
__device__ inline void label_row(const float* __restrict__ P, const float* __restrict__ my,
                                 const float* __restrict__ sy, int q, double* __restrict__ out) {
  double U[kNetMaxQ * kNetMaxQ];
  for (int c = 0; c < 1 + q; ++c) out[c] = (double)P[c] * (double)sy[c] + (double)my[c];
  int c = 1 + q;
  for (int a = 0; a < q; ++a)
    for (int b = a; b < q; ++b, ++c) {
      const double v = (double)P[c] * (double)sy[c] + (double)my[c];
      U[a * q + b] = (a == b) ? exp(v) : v;
    }
  c = 1 + q;
  for (int a = 0; a < q; ++a)
    for (int b = a; b < q; ++b, ++c) {
      double cov = 0.0;
      for (int k = 0; k <= a; ++k) cov += U[k * q + a] * U[k * q + b];
      out[c] = cov + out[1 + a] * out[1 + b];
    }
}

// label rows -> network rows, one thread per row
__global__ void net_targets_kernel(const double* __restrict__ targ, int64_t M, int q, int OUT,
                                   double* __restrict__ out) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= M) return;
  net_row(targ + r * OUT, q, out + r * OUT);
}

// Standardised, padded rows: X[r] = (feat[idx[r]] - mx) / sx in bf16 (width
// 64) and, when targ (network rows) is given, T[r] = (targ[idx[r]] - my) / sy
// (fp32, width OUT).  Rows r >= B (padding to a multiple of 64) are zero;
// idx NULL means row base + r.
__global__ void gather_rows_kernel(const double* __restrict__ feat, const double* __restrict__ targ,
                                   const int64_t* __restrict__ idx, int64_t base, int64_t B,
                                   int64_t Bp, int IN, int OUT, const float* __restrict__ mx,
                                   const float* __restrict__ sx, const float* __restrict__ my,
                                   const float* __restrict__ sy, bf16* __restrict__ X,
                                   float* __restrict__ T) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= Bp * kMlpPad) return;
  const int64_t r = t / kMlpPad;
  const int c = (int)(t % kMlpPad);
  const int64_t s = r < B ? (idx ? idx[base + r] : base + r) : 0;
  float xv = 0.f;
  if (r < B && c < IN) xv = (float)((feat[s * IN + c] - (double)mx[c]) / (double)sx[c]);
  X[t] = f2bf(xv);
  if (targ && c < OUT) {
    float tv = 0.f;
    if (r < B) tv = (float)((targ[s * OUT + c] - (double)my[c]) / (double)sy[c]);
    T[r * OUT + c] = tv;
  }
}

// network outputs of rows r < B back to label rows (double), one thread per row
__global__ void unstd_kernel(const float* __restrict__ P, int64_t B, int OUT, int q,
                             const float* __restrict__ my, const float* __restrict__ sy,
                             double* __restrict__ out) {
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= B) return;
  label_row(P + r * kMlpPad, my, sy, q, out + r * OUT);
}

}  // namespace
}  // namespace cfust
