// C ABI of the surrogate form: the network handle (parameters, optimiser
// state, standardisation), its training and inference on the matrix cores,
// run-time adaptation, the surrogate E-step pairs with the GHK fallback, GHK
// label batches and the pair features.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/cfust.h"
#include "cfust_host.hpp"
#include "cfust_surrogate.hpp"

using namespace cfust;
using namespace cfust::host;

// Surrogate network handle: parameters, optimiser state and standardisation
// on the device, plus the inference and training buffers it grows on demand.
struct cfust_surrogate {
  int q = 0, F = 0, T = 0;
  SurrRange rg{};
  float* params = nullptr;  // [kMlpParams] fp32 master weights
  float* grad = nullptr;    // [kMlpParams]
  float* adm = nullptr;     // Adam first moments
  float* adv = nullptr;     // Adam second moments
  bf16* wb = nullptr;       // [kMlpWeightsBf] bf16 weights
  float* stdv = nullptr;    // [CFUST_SURR_STD] device standardisation
  float* wo = nullptr;      // [64] loss weights per output
  float h_std[CFUST_SURR_STD];
  bool have_std = false;
  int64_t adam_t = 0;
  int em_switch = -1;                      // first GHK E-step of the last cfust_em_fit
  hipStream_t own = nullptr;               // training stream (capturable)
  int64_t* dstep = nullptr;                // device step counter of a training run
  unsigned long long* fb_total = nullptr;  // device: fallback pairs of the last E-step
  // inference buffers (pairs per chunk)
  int64_t cap_pairs = 0;
  bf16* X = nullptr;
  float* P = nullptr;
  unsigned char* inr = nullptr;
  int64_t* list = nullptr;
  unsigned int* count = nullptr;
  float* cf = nullptr;
  int* cok = nullptr;
  // training buffers (rows per minibatch)
  int64_t cap_rows = 0;
  bf16 *tX = nullptr, *tH[3] = {}, *tdPb = nullptr, *tdPlo = nullptr, *tdZb[2] = {},
       *tdZlo[2] = {};
  float *tT = nullptr, *tZ[3] = {}, *tP = nullptr, *tdP = nullptr, *tdZ[2] = {}, *tpart = nullptr,
        *tbpart = nullptr, *tloss = nullptr;
};

namespace {

// ---------------------------------------------------------------------------
// surrogate network: matrix-core products and the forward pass
// ---------------------------------------------------------------------------
int64_t round64(int64_t x) { return (x + 63) / 64 * 64; }

// M (rows) on grid x, N / 64 column tiles on grid y, K split over grid z
template <bool TA, bool TB, int MODE, bool SPLIT = false>
void gemm(const bf16* A, const bf16* A2, int lda, const bf16* B, int ldb, int64_t M, int N, int K,
          int splits, Epi ep, hipStream_t st) {
  int kps = K;
  if (splits > 1) {
    kps = ((K + splits - 1) / splits + 31) / 32 * 32;
    splits = (K + kps - 1) / kps;
  } else {
    splits = 1;
  }
  dim3 grid((unsigned)(M / 64), (unsigned)(N / 64), (unsigned)splits);
  gemm_bf16_kernel<TA, TB, MODE, SPLIT><<<grid, 256, 0, st>>>(A, A2, lda, B, ldb, (int)M, N, K,
                                                               kps, ep);
}

// rows (multiple of 64) through the four layers: X -> H[0] -> H[1] -> H[2] ->
// P (fp32, 64 wide); pre-activations kept in Z when given (training)
void mlp_forward(const cfust_surrogate* s, const bf16* X, int64_t rows, bf16* const H[3],
                 float* const* Z, float* P, hipStream_t st) {
  const bf16* in = X;
  for (int l = 0; l < kMlpLayers; ++l) {
    const int K = mlp_k(l), N = mlp_n(l);
    Epi ep{};
    ep.b = s->params + mlp_b_off(l);
    if (l < kMlpLayers - 1) {
      ep.H = H[l];
      ep.Zs = Z ? Z[l] : nullptr;
      ep.ldc = N;
      gemm<false, true, kEpiBiasSilu>(in, nullptr, K, s->wb + mlp_wb_off(l), K, rows, N, K, 1, ep,
                                      st);
      in = H[l];
    } else {
      ep.C = P;
      ep.ldc = N;
      gemm<false, true, kEpiBias>(in, nullptr, K, s->wb + mlp_wb_off(l), K, rows, N, K, 1, ep, st);
    }
  }
}

// inference: all four layers in one kernel per 16 kInferRT rows (the last
// block ragged)
void mlp_infer(const cfust_surrogate* s, const bf16* X, int64_t rows, float* P, hipStream_t st) {
  constexpr int R = 16 * kInferRT;
  if (rows > 0)
    mlp_infer_kernel<kInferRT><<<(unsigned)((rows + R - 1) / R), 256, 0, st>>>(X, rows, s->wb,
                                                                              s->params, P);
}

template <typename X>
bool dev_alloc(X** p, size_t count) {
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  return hipMalloc((void**)p, count * sizeof(X) + 256) == hipSuccess;
}

// inference buffers for `pairs` pairs per chunk (two feature rows each)
int ensure_infer(cfust_surrogate* s, int64_t pairs) {
  if (pairs <= s->cap_pairs) return CFUST_OK;
  const int64_t rows = round64(2 * pairs);
  bool ok = dev_alloc(&s->X, rows * kMlpPad) && dev_alloc(&s->P, rows * kMlpPad) &&
            dev_alloc(&s->inr, pairs) && dev_alloc(&s->list, pairs);
  if (!ok) {
    s->cap_pairs = 0;
    return CFUST_ENOMEM;
  }
  s->cap_pairs = pairs;
  return CFUST_OK;
}

constexpr int64_t kSurrChunkPairs = int64_t(1) << 19;

}  // namespace

namespace cfust {
namespace host {

// E-step pairs through the network; pairs outside the training range through
// the GHK kernel (on a compacted list per chunk)
template <typename T, int Q, int PM>
int launch_surrogate_pairs_q(const Ws& ws, const Plan& pl, const double* y, const double* mu) {
  cfust_surrogate* s = ws.surr;
  const int64_t pairs = pl.n * pl.g;
  if (pairs == 0) return CFUST_OK;
  const int64_t chunk = std::min(pairs, kSurrChunkPairs);
  int rc = ensure_infer(s, chunk);
  if (rc) return rc;
  const double* comp = ws.at<double>(pl.o_comp);
  int* status = ws.at<int>(pl.o_status);
  surr_comp_kernel<<<1, 64, 0, ws.st>>>(pl.p, pl.q, pl.g, comp, s->rg, s->stdv, s->cf, s->cok);
  fill_u64_kernel<<<1, 64, 0, ws.st>>>(s->fb_total, 0ull);
  for (int64_t c0 = 0; c0 < pairs; c0 += chunk) {
    const int64_t cn = std::min(chunk, pairs - c0);
    const unsigned nb = (unsigned)((cn + 255) / 256);
    fill_uint_kernel<<<1, 64, 0, ws.st>>>(s->count, 0u);
    surr_feat_kernel<Q, PM><<<nb, 256, 0, ws.st>>>(y, pl.p, pl.g, mu, comp, c0, cn, s->rg, s->stdv,
                                               s->cf, s->cok, s->X, s->inr, s->list, s->count,
                                               status);
    mlp_infer(s, s->X, round64(2 * cn), s->P, ws.st);
    surr_assemble_kernel<Q, PM><<<nb, 256, 0, ws.st>>>(y, pl.p, pl.g, mu, comp, c0, cn, s->P,
                                                   s->stdv, s->inr, ws.at<double>(pl.o_pair),
                                                   pl.W);
    const unsigned lb = (unsigned)std::min<int64_t>((cn + 3) / 4, 8192);
    pair_list_kernel<T, Q><<<lb, 256, 0, ws.st>>>(
        y, pl.p, pl.g, mu, comp, ws.at<T>(pl.o_sA), ws.at<T>(pl.o_sB), ws.at<T>(pl.o_rsB),
        ws.at<T>(pl.o_uT), ws.at<T>(pl.o_ubT), pl.N, s->list, s->count, ws.at<double>(pl.o_pair),
        pl.W, status);
    add_count_kernel<<<1, 64, 0, ws.st>>>(s->count, s->fb_total);
  }
  return CFUST_OK;
}

template <typename T, int PM>
int launch_surrogate_pairs_p(const Ws& ws, const Plan& pl, const double* y, const double* mu) {
  switch (pl.q) {
    case 1: return launch_surrogate_pairs_q<T, 1, PM>(ws, pl, y, mu);
    case 2: return launch_surrogate_pairs_q<T, 2, PM>(ws, pl, y, mu);
    case 3: return launch_surrogate_pairs_q<T, 3, PM>(ws, pl, y, mu);
    case 4: return launch_surrogate_pairs_q<T, 4, PM>(ws, pl, y, mu);
    case 5: return launch_surrogate_pairs_q<T, 5, PM>(ws, pl, y, mu);
    case 6: return launch_surrogate_pairs_q<T, 6, PM>(ws, pl, y, mu);
    case 7: return launch_surrogate_pairs_q<T, 7, PM>(ws, pl, y, mu);
    case 8: return launch_surrogate_pairs_q<T, 8, PM>(ws, pl, y, mu);
  }
  return CFUST_EINVAL;
}

// thread-per-pair kernels keep p-vectors in registers for p <= 8
template <typename T>
int launch_surrogate_pairs(const Ws& ws, const Plan& pl, const double* y, const double* mu) {
  if (pl.p <= 8) return launch_surrogate_pairs_p<T, 8>(ws, pl, y, mu);
  return launch_surrogate_pairs_p<T, kMaxP>(ws, pl, y, mu);
}

template int launch_surrogate_pairs<double>(const Ws&, const Plan&, const double*, const double*);
template int launch_surrogate_pairs<float>(const Ws&, const Plan&, const double*, const double*);

bool surrogate_ready(const cfust_surrogate* s, int q) { return s && s->q == q && s->have_std; }

void surrogate_set_switch(cfust_surrogate* s, int t) {
  if (s) s->em_switch = t;
}

}  // namespace host
}  // namespace cfust

// ===========================================================================
// GHK integrals for a batch of standardised problems
// ===========================================================================
namespace {

template <typename T, int Q>
void launch_ghk_batch_q(int64_t M, const double* h, const double* R, const int* tab, char* base,
                        size_t o_s, size_t o_rs, size_t o_uT, size_t o_ubT, int N, double* out,
                        int* status, hipStream_t st) {
  ghk_batch_kernel<T, Q><<<(unsigned)((M + 3) / 4), 256, 0, st>>>(
      M, h, R, tab, (const T*)(base + o_s), (const T*)(base + o_rs), (const T*)(base + o_uT),
      (const T*)(base + o_ubT), N, out, status);
}

template <typename T>
int run_ghk_batch(int q, int64_t M, const double* h, const double* R, const double* dof,
                  const double* u, int N, double* out, hipStream_t st) {
  // distinct degrees of freedom (host) -> one table pair each
  std::vector<double> hd((size_t)M);
  if (hipMemcpyAsync(hd.data(), dof, M * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return CFUST_EHIP;
  std::vector<double> uniq(hd);
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  if (uniq.size() > 4096) return CFUST_EINVAL;
  std::vector<int> tab((size_t)M);
  for (int64_t s = 0; s < M; ++s)
    tab[s] = (int)(std::lower_bound(uniq.begin(), uniq.end(), hd[s]) - uniq.begin());
  const int nd = (int)uniq.size();
  const size_t es = sizeof(T);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  size_t o_status = take(4 * sizeof(int));
  size_t o_d = take(nd * sizeof(double));
  size_t o_tab = take(M * sizeof(int));
  size_t o_s = take((size_t)nd * N * es);
  size_t o_rs = take((size_t)nd * N * es);
  size_t o_uT = take((size_t)(q + 1) * N * es);
  size_t o_ubT = take((size_t)(q + 1) * N * es);
  char* base = nullptr;
  if (hipMallocAsync((void**)&base, off, st) != hipSuccess) return CFUST_ENOMEM;
  int* status = (int*)(base + o_status);
  fill_int_kernel<<<1, 64, 0, st>>>(status, 4, 0);
  (void)hipMemcpyAsync(base + o_d, uniq.data(), nd * sizeof(double), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(base + o_tab, tab.data(), M * sizeof(int), hipMemcpyHostToDevice, st);
  int64_t tot = (int64_t)N * (q + 1);
  points_kernel<T><<<(unsigned)((tot + 255) / 256), 256, 0, st>>>(u, N, q + 1, (T*)(base + o_uT),
                                                                  (T*)(base + o_ubT), status);
  int64_t tq = (int64_t)nd * N;
  chi_list_kernel<T><<<(unsigned)((tq + 127) / 128), 128, 0, st>>>(
      (const double*)(base + o_d), nd, u, N, q + 1, (T*)(base + o_s), (T*)(base + o_rs), status);
  const int* tb = (const int*)(base + o_tab);
  switch (q) {
    case 1: launch_ghk_batch_q<T, 1>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 2: launch_ghk_batch_q<T, 2>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 3: launch_ghk_batch_q<T, 3>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 4: launch_ghk_batch_q<T, 4>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 5: launch_ghk_batch_q<T, 5>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 6: launch_ghk_batch_q<T, 6>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 7: launch_ghk_batch_q<T, 7>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
    case 8: launch_ghk_batch_q<T, 8>(M, h, R, tb, base, o_s, o_rs, o_uT, o_ubT, N, out, status, st); break;
  }
  int rc = launch_check();
  int hs[2] = {0, 0};
  (void)hipMemcpyAsync(hs, status, 2 * sizeof(int), hipMemcpyDeviceToHost, st);
  if (hipStreamSynchronize(st) != hipSuccess) rc = CFUST_EHIP;
  (void)hipFreeAsync(base, st);
  (void)hipStreamSynchronize(st);
  if (rc) return rc;
  if (hs[0] == kOk) return CFUST_OK;
  return hs[0] == kENotPD ? CFUST_ENOTPD : CFUST_EINVAL;
}

}  // namespace

extern "C" int cfust_ghk_batch(int q, int64_t M, const double* h, const double* R,
                               const double* dof, const double* u, int n_qmc, const cfust_opts* o,
                               double* out) {
  if (q < 1 || q > kMaxQFull || M < 0 || n_qmc < 1 || (M > 0 && (!h || !R || !dof || !out)) || !u)
    return CFUST_EINVAL;
  int rc = check_opts(o);
  if (rc) return rc;
  if (o && o->reorder) return CFUST_EINVAL;
  if (M == 0) return CFUST_OK;
  hipStream_t st = o ? (hipStream_t)o->stream : nullptr;
  if (o && o->precision == CFUST_FP32) return run_ghk_batch<float>(q, M, h, R, dof, u, n_qmc, out, st);
  return run_ghk_batch<double>(q, M, h, R, dof, u, n_qmc, out, st);
}

// ===========================================================================
// surrogate network: handle, training, inference
// ===========================================================================
namespace {

// splitmix64 (Steele, Lea & Flood 2014) and Box-Muller normals for the
// weight initialisation and the minibatch shuffles
struct Rng {
  unsigned long long x;
  unsigned long long next() {
    unsigned long long z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u1 = uniform(), u2 = uniform();
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
};

int surr_feat_width(int q) { return q + q * (q - 1) / 2 + 1; }
int surr_targ_width(int q) { return 1 + q + q * (q + 1) / 2; }

void free_surrogate(cfust_surrogate* s) {
  void* ptrs[] = {s->params, s->grad, s->adm,   s->adv,  s->wb,    s->stdv,  s->wo,
                  s->fb_total, s->X,  s->P,     s->inr,   s->list,
                  s->count,  s->cf,   s->cok,   s->tX,   s->tH[0], s->tH[1], s->tH[2],
                  s->tdPb,   s->tdZb[0], s->tdZb[1], s->tT, s->tZ[0], s->tZ[1], s->tZ[2],
                  s->tdPlo,  s->tdZlo[0], s->tdZlo[1],
                  s->tP,     s->tdP,  s->tdZ[0], s->tdZ[1], s->tpart, s->tbpart, s->tloss};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (s->dstep) (void)hipFree(s->dstep);
  if (s->own) (void)hipStreamDestroy(s->own);
  delete s;
}

int refresh_bf16(cfust_surrogate* s, hipStream_t st) {
  weights_to_bf16_kernel<<<(unsigned)((kMlpWeightsBf + 255) / 256), 256, 0, st>>>(s->params, s->wb);
  return launch_check();
}

// buffers of one training minibatch of `rows` rows (multiple of 64)
int ensure_train(cfust_surrogate* s, int64_t rows) {
  if (rows <= s->cap_rows) return CFUST_OK;
  bool ok = dev_alloc(&s->tX, rows * kMlpPad) && dev_alloc(&s->tT, rows * kMlpPad) &&
            dev_alloc(&s->tP, rows * kMlpPad) && dev_alloc(&s->tdP, rows * kMlpPad) &&
            dev_alloc(&s->tdPb, rows * kMlpPad) && dev_alloc(&s->tdPlo, rows * kMlpPad) &&
            dev_alloc(&s->tpart, (size_t)256 * 4096) &&
            dev_alloc(&s->tbpart, (size_t)(rows / 256 + 1) * kMlpHid) &&
            dev_alloc(&s->tloss, rows * kMlpPad / 256 + 1);
  for (int l = 0; l < 3 && ok; ++l)
    ok = dev_alloc(&s->tH[l], rows * kMlpHid) && dev_alloc(&s->tZ[l], rows * kMlpHid);
  for (int l = 0; l < 2 && ok; ++l)
    ok = dev_alloc(&s->tdZ[l], rows * kMlpHid) && dev_alloc(&s->tdZb[l], rows * kMlpHid) &&
         dev_alloc(&s->tdZlo[l], rows * kMlpHid);
  if (!ok) {
    s->cap_rows = 0;
    return CFUST_ENOMEM;
  }
  s->cap_rows = rows;
  return CFUST_OK;
}

// column sums of X[rows][N] into out[N]
void colsum(cfust_surrogate* s, const float* X, int64_t rows, int N, float* out, hipStream_t st) {
  const unsigned chunks = (unsigned)((rows + 255) / 256);
  colsum_part_kernel<<<dim3(N / 64, chunks), 256, 0, st>>>(X, rows, N, s->tbpart);
  sum_slices_kernel<<<(N + 255) / 256, 256, 0, st>>>(s->tbpart, (int)chunks, N, out);
}

// dW (fp32, [N_out][K_in]) = dZ^T H over `rows` rows (dZ as high and low
// bf16 parts), split over the rows
void weight_grad(cfust_surrogate* s, const bf16* dZb, const bf16* dZlo, int n_out,
                 const bf16* Hin, int k_in, int64_t rows, float* out, hipStream_t st) {
  const int tiles = (n_out / 64) * (k_in / 64);
  int splits = (int)std::max<int64_t>(1, std::min<int64_t>(256 / tiles, rows / 128));
  int kps = (int)((rows + splits - 1) / splits + 31) / 32 * 32;
  splits = (int)((rows + kps - 1) / kps);
  Epi ep{};
  ep.C = s->tpart;
  ep.ldc = k_in;
  dim3 grid((unsigned)(n_out / 64), (unsigned)(k_in / 64), (unsigned)splits);
  gemm_bf16_kernel<true, false, kEpiStore, true><<<grid, 256, 0, st>>>(
      dZb, dZlo, n_out, Hin, k_in, n_out, k_in, (int)rows, kps, ep);
  const int64_t n = (int64_t)n_out * k_in;
  sum_slices_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(s->tpart, splits, n, out);
}

// one minibatch already gathered into tX / tT (Bp rows, B valid): forward,
// loss (added to lacc[slot], or lacc[*dstep / per_epoch] when dstep is given)
// and gradient into s->grad
void forward_backward(cfust_surrogate* s, int64_t B, int64_t Bp, float wsum, double* lacc,
                      int slot, hipStream_t st, const int64_t* dstep = nullptr,
                      int64_t per_epoch = 1) {
  mlp_forward(s, s->tX, Bp, s->tH, s->tZ, s->tP, st);
  const unsigned nlb = (unsigned)(Bp * kMlpPad / 256);
  mse_grad_kernel<<<nlb, 256, 0, st>>>(s->tP, s->tT, Bp, B, s->T, s->wo, wsum, s->tdP, s->tdPb,
                                       s->tdPlo, s->tloss);
  if (dstep)
    accumulate_step_kernel<<<1, 256, 0, st>>>(s->tloss, (int)nlb, lacc, dstep, per_epoch);
  else
    accumulate_kernel<<<1, 256, 0, st>>>(s->tloss, (int)nlb, lacc, slot);
  // layer 3 (linear output)
  weight_grad(s, s->tdPb, s->tdPlo, kMlpPad, s->tH[2], kMlpHid, Bp, s->grad + mlp_w_off(3), st);
  colsum(s, s->tdP, Bp, kMlpPad, s->grad + mlp_b_off(3), st);
  const bf16* dzb = s->tdPb;
  const bf16* dzlo = s->tdPlo;
  int nout = kMlpPad;
  int cur = 0;
  for (int l = 2; l >= 0; --l) {
    // dZ_l = (dZ_{l+1} W_{l+1}) * SiLU'(Z_l)
    Epi ep{};
    ep.C = s->tdZ[cur];
    ep.Zs = s->tZ[l];
    ep.H = s->tdZb[cur];
    ep.H2 = s->tdZlo[cur];
    ep.ldc = kMlpHid;
    gemm<false, false, kEpiSiluBwd, true>(dzb, dzlo, nout, s->wb + mlp_wb_off(l + 1), kMlpHid, Bp,
                                          kMlpHid, nout, 1, ep, st);
    const bf16* hin = l > 0 ? s->tH[l - 1] : s->tX;
    const int kin = mlp_k(l);
    weight_grad(s, s->tdZb[cur], s->tdZlo[cur], kMlpHid, hin, kin, Bp, s->grad + mlp_w_off(l), st);
    colsum(s, s->tdZ[cur], Bp, kMlpHid, s->grad + mlp_b_off(l), st);
    dzb = s->tdZb[cur];
    dzlo = s->tdZlo[cur];
    nout = kMlpHid;
    cur ^= 1;
  }
}

float set_loss_weights(cfust_surrogate* s, const float* wo, hipStream_t st) {
  float h[kMlpPad];
  float sum = 0.f;
  for (int o = 0; o < kMlpPad; ++o) {
    h[o] = o < s->T ? (wo ? wo[o] : 1.0f) : 0.0f;
    sum += h[o];
  }
  (void)hipMemcpyAsync(s->wo, h, sizeof(h), hipMemcpyHostToDevice, st);
  (void)hipStreamSynchronize(st);
  return sum;
}

// label rows -> network rows in a stream-ordered temporary (caller frees)
int network_rows(cfust_surrogate* s, const double* targ, int64_t M, hipStream_t st, double** nt) {
  *nt = nullptr;
  if (hipMallocAsync((void**)nt, (size_t)M * s->T * sizeof(double), st) != hipSuccess)
    return CFUST_ENOMEM;
  net_targets_kernel<<<(unsigned)((M + 255) / 256), 256, 0, st>>>(targ, M, s->q, s->T, *nt);
  return launch_check();
}

// standardisation from features and network rows
int set_std_from_data(cfust_surrogate* s, const double* feat, const double* nt, int64_t M,
                      hipStream_t st) {
  col_moments_kernel<<<s->F, 256, 0, st>>>(feat, M, s->F, s->stdv, s->stdv + kMlpPad);
  col_moments_kernel<<<s->T, 256, 0, st>>>(nt, M, s->T, s->stdv + 2 * kMlpPad,
                                           s->stdv + 3 * kMlpPad);
  if (hipMemcpyAsync(s->h_std, s->stdv, sizeof(s->h_std), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return CFUST_EHIP;
  s->have_std = true;
  return CFUST_OK;
}

template <int PM>
void launch_pair_features(int q, unsigned nb, hipStream_t st, const double* y, int64_t n, int p,
                          int g, const double* mu, const double* comp, double* out, int* status) {
  switch (q) {
    case 1: pair_features_kernel<1, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 2: pair_features_kernel<2, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 3: pair_features_kernel<3, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 4: pair_features_kernel<4, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 5: pair_features_kernel<5, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 6: pair_features_kernel<6, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 7: pair_features_kernel<7, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
    case 8: pair_features_kernel<8, PM><<<nb, 128, 0, st>>>(y, n, p, g, mu, comp, out, status); break;
  }
}

template <int PM>
void launch_features_list(int q, unsigned nb, hipStream_t st, const double* y, int p, int g,
                          const double* mu, const double* comp, const int64_t* pick, int64_t m,
                          double* out, int* status) {
  switch (q) {
    case 1: pair_features_list_kernel<1, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 2: pair_features_list_kernel<2, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 3: pair_features_list_kernel<3, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 4: pair_features_list_kernel<4, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 5: pair_features_list_kernel<5, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 6: pair_features_list_kernel<6, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 7: pair_features_list_kernel<7, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
    case 8: pair_features_list_kernel<8, PM><<<nb, 128, 0, st>>>(y, p, g, mu, comp, pick, m, out, status); break;
  }
}

struct SurrFileHeader {
  char magic[8];
  int32_t version, q, F, T, hidden, layers;
  int64_t nparams;
  double range[6];
};

}  // namespace

extern "C" {

int cfust_surrogate_create(int q, const double* range, unsigned long long seed,
                           cfust_surrogate** out) {
  if (!out || !range || q < 1 || q > kMaxQFull) return CFUST_EINVAL;
  *out = nullptr;
  if (!(range[0] < range[1]) || !(range[2] > 0.0) || !(range[2] <= range[3]) ||
      !(range[4] > 0.0) || !(range[5] >= 0.0))
    return CFUST_EINVAL;
  static_assert(kMlpParams == CFUST_SURR_PARAMS, "parameter count");
  cfust_surrogate* s = new cfust_surrogate;
  s->q = q;
  s->F = surr_feat_width(q);
  s->T = surr_targ_width(q);
  s->rg = SurrRange{range[0], range[1], range[2], range[3], range[4], range[5]};
  bool ok = dev_alloc(&s->params, kMlpParams) && dev_alloc(&s->grad, kMlpParams) &&
            dev_alloc(&s->adm, kMlpParams) && dev_alloc(&s->adv, kMlpParams) &&
            dev_alloc(&s->wb, kMlpWeightsBf) && dev_alloc(&s->stdv, CFUST_SURR_STD) &&
            dev_alloc(&s->wo, kMlpPad) && dev_alloc(&s->fb_total, 1) &&
            dev_alloc(&s->count, 1) && dev_alloc(&s->cf, kMaxG * 32) && dev_alloc(&s->cok, kMaxG) &&
            dev_alloc(&s->dstep, 1) &&
            hipStreamCreateWithFlags(&s->own, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    free_surrogate(s);
    return CFUST_ENOMEM;
  }
  std::vector<float> w((size_t)kMlpParams, 0.0f);
  Rng rng{seed};
  for (int l = 0; l < kMlpLayers; ++l) {
    const int kv = l == 0 ? s->F : kMlpHid;          // fan-in without padding
    const int nv = l == kMlpLayers - 1 ? s->T : kMlpHid;
    const double sd = l == kMlpLayers - 1 ? sqrt(1.0 / kv) : sqrt(2.0 / kv);
    for (int o = 0; o < nv; ++o)
      for (int i = 0; i < kv; ++i) w[mlp_w_off(l) + (int64_t)o * mlp_k(l) + i] = (float)(sd * rng.normal());
  }
  for (int c = 0; c < CFUST_SURR_STD; ++c) s->h_std[c] = (c / kMlpPad) % 2 == 1 ? 1.0f : 0.0f;
  ok = hipMemcpy(s->params, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice) ==
           hipSuccess &&
       hipMemset(s->adm, 0, kMlpParams * sizeof(float)) == hipSuccess &&
       hipMemset(s->adv, 0, kMlpParams * sizeof(float)) == hipSuccess &&
       hipMemset(s->fb_total, 0, sizeof(unsigned long long)) == hipSuccess &&
       hipMemcpy(s->stdv, s->h_std, sizeof(s->h_std), hipMemcpyHostToDevice) == hipSuccess;
  if (ok) {
    set_loss_weights(s, nullptr, nullptr);
    ok = refresh_bf16(s, nullptr) == CFUST_OK && hipDeviceSynchronize() == hipSuccess;
  }
  if (!ok) {
    free_surrogate(s);
    return CFUST_EHIP;
  }
  *out = s;
  return CFUST_OK;
}

void cfust_surrogate_destroy(cfust_surrogate* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  free_surrogate(s);
}

int cfust_surrogate_train(cfust_surrogate* s, const double* feat, const double* targ, int64_t M,
                          int epochs, int batch, double lr0, double lr1, unsigned long long seed,
                          const float* wo, const cfust_opts* o, double* loss_trace) {
  if (!s || !feat || !targ || M < 1 || epochs < 0 || batch < 64 || batch % 64 || batch > 65536 ||
      !(lr0 > 0.0) || !(lr1 >= 0.0))
    return CFUST_EINVAL;
  hipStream_t st = o ? (hipStream_t)o->stream : nullptr;
  int rc = ensure_train(s, batch);
  if (rc) return rc;
  double* nt = nullptr;
  if ((rc = network_rows(s, targ, M, st, &nt))) {
    if (nt) (void)hipFreeAsync(nt, st);
    return rc;
  }
  if (!s->have_std && (rc = set_std_from_data(s, feat, nt, M, st))) {
    (void)hipFreeAsync(nt, st);
    return rc;
  }
  const float wsum = set_loss_weights(s, wo, st);
  int64_t* idx = nullptr;
  double* lacc = nullptr;
  if (!(wsum > 0.f) || hipMallocAsync((void**)&idx, M * sizeof(int64_t), st) != hipSuccess) {
    (void)hipFreeAsync(nt, st);
    return wsum > 0.f ? CFUST_ENOMEM : CFUST_EINVAL;
  }
  if (hipMallocAsync((void**)&lacc, (epochs + 1) * sizeof(double), st) != hipSuccess) {
    (void)hipFreeAsync(idx, st);
    (void)hipFreeAsync(nt, st);
    return CFUST_ENOMEM;
  }
  (void)hipMemsetAsync(lacc, 0, (epochs + 1) * sizeof(double), st);
  // The run goes on the handle's own stream (capturable): every step is the
  // same launch sequence reading its minibatch offset, loss slot and Adam
  // step from the device counter s->dstep; with opts->graph (default) it is
  // captured once and replayed.  Each epoch takes floor(M / B) minibatches of
  // B = min(batch, M) rows of a fresh shuffle.
  if (hipStreamSynchronize(st) != hipSuccess) rc = CFUST_EHIP;
  hipStream_t ow = s->own;
  const int64_t B = std::min<int64_t>(batch, M);
  const int64_t Bp = round64(B);
  const int64_t steps = M / B;
  const int64_t total = steps * (int64_t)epochs;
  TrainStep ts{s->dstep, steps, total, B, Bp, s->adam_t, lr0, lr1};
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  auto one_step = [&]() {
    gather_step_kernel<<<(unsigned)(Bp * kMlpPad / 256), 256, 0, ow>>>(
        feat, nt, idx, ts, s->F, s->T, s->stdv, s->stdv + kMlpPad, s->stdv + 2 * kMlpPad,
        s->stdv + 3 * kMlpPad, s->tX, s->tT);
    forward_backward(s, B, Bp, wsum, lacc, 0, ow, s->dstep, steps);
    adam_step_kernel<<<(unsigned)((kMlpParams + 255) / 256), 256, 0, ow>>>(
        s->params, s->grad, s->adm, s->adv, kMlpParams, ts, b1, b2, eps);
    weights_to_bf16_kernel<<<(unsigned)((kMlpWeightsBf + 255) / 256), 256, 0, ow>>>(s->params,
                                                                                    s->wb);
    step_inc_kernel<<<1, 64, 0, ow>>>(s->dstep);
  };
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const bool use_graph = !o || o->graph;
  if (!rc && hipMemsetAsync(s->dstep, 0, sizeof(int64_t), ow) != hipSuccess) rc = CFUST_EHIP;
  if (!rc && use_graph && total > 0) {
    if (hipStreamBeginCapture(ow, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      rc = CFUST_EHIP;
    } else {
      one_step();
      if (hipStreamEndCapture(ow, &graph) != hipSuccess ||
          hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
        rc = CFUST_EHIP;
    }
  }
  std::vector<int64_t> perm((size_t)M);
  Rng rng{seed};
  for (int ep = 0; ep < epochs && !rc; ++ep) {
    for (int64_t k = 0; k < M; ++k) perm[k] = k;
    for (int64_t k = M - 1; k > 0; --k) std::swap(perm[k], perm[rng.next() % (uint64_t)(k + 1)]);
    if (hipMemcpyAsync(idx, perm.data(), M * sizeof(int64_t), hipMemcpyHostToDevice, ow) !=
        hipSuccess) {
      rc = CFUST_EHIP;
      break;
    }
    for (int64_t k = 0; k < steps; ++k) {
      if (exec) {
        if (hipGraphLaunch(exec, ow) != hipSuccess) {
          rc = CFUST_EHIP;
          break;
        }
      } else {
        one_step();
      }
    }
    if (!rc) rc = launch_check();
    // the host permutation is rewritten next epoch: wait for the upload
    if (hipStreamSynchronize(ow) != hipSuccess && !rc) rc = CFUST_EHIP;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (hipStreamSynchronize(ow) != hipSuccess && !rc) rc = CFUST_EHIP;
  if (!rc) s->adam_t += total;
  if (!rc && loss_trace && epochs > 0) {
    std::vector<double> h((size_t)epochs);
    if (hipMemcpyAsync(h.data(), lacc, epochs * sizeof(double), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = CFUST_EHIP;
    for (int e = 0; e < epochs; ++e) loss_trace[e] = h[e] / (double)steps;
  }
  (void)hipFreeAsync(idx, st);
  (void)hipFreeAsync(lacc, st);
  (void)hipFreeAsync(nt, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = CFUST_EHIP;
  return rc;
}

int cfust_surrogate_grad(cfust_surrogate* s, const double* feat, const double* targ, int64_t M,
                         const float* wo, const cfust_opts* o, float* grad, double* loss) {
  if (!s || !feat || !targ || !grad || !loss || M < 1 || M > 65536 || !s->have_std)
    return CFUST_EINVAL;
  hipStream_t st = o ? (hipStream_t)o->stream : nullptr;
  const int64_t Bp = round64(M);
  int rc = ensure_train(s, Bp);
  if (rc) return rc;
  const float wsum = set_loss_weights(s, wo, st);
  if (!(wsum > 0.f)) return CFUST_EINVAL;
  double* nt = nullptr;
  if ((rc = network_rows(s, targ, M, st, &nt))) {
    if (nt) (void)hipFreeAsync(nt, st);
    return rc;
  }
  double* lacc = nullptr;
  if (hipMallocAsync((void**)&lacc, sizeof(double), st) != hipSuccess) {
    (void)hipFreeAsync(nt, st);
    return CFUST_ENOMEM;
  }
  (void)hipMemsetAsync(lacc, 0, sizeof(double), st);
  gather_rows_kernel<<<(unsigned)(Bp * kMlpPad / 256), 256, 0, st>>>(
      feat, nt, nullptr, 0, M, Bp, s->F, s->T, s->stdv, s->stdv + kMlpPad, s->stdv + 2 * kMlpPad,
      s->stdv + 3 * kMlpPad, s->tX, s->tT);
  forward_backward(s, M, Bp, wsum, lacc, 0, st);
  rc = launch_check();
  if (!rc && (hipMemcpyAsync(grad, s->grad, kMlpParams * sizeof(float), hipMemcpyDeviceToHost,
                             st) != hipSuccess ||
              hipMemcpyAsync(loss, lacc, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess))
    rc = CFUST_EHIP;
  (void)hipFreeAsync(lacc, st);
  (void)hipFreeAsync(nt, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = CFUST_EHIP;
  return rc;
}

int cfust_surrogate_eval(cfust_surrogate* s, const double* feat, int64_t M, const cfust_opts* o,
                         double* out) {
  if (!s || M < 0 || (M > 0 && (!feat || !out)) || !s->have_std) return CFUST_EINVAL;
  if (M == 0) return CFUST_OK;
  hipStream_t st = o ? (hipStream_t)o->stream : nullptr;
  const int64_t chunk_rows = 2 * kSurrChunkPairs;
  int rc = ensure_infer(s, std::min<int64_t>(kSurrChunkPairs, (M + 1) / 2));
  if (rc) return rc;
  for (int64_t r0 = 0; r0 < M; r0 += chunk_rows) {
    const int64_t B = std::min(chunk_rows, M - r0);
    const int64_t Bp = round64(B);
    gather_rows_kernel<<<(unsigned)(Bp * kMlpPad / 256), 256, 0, st>>>(
        feat, nullptr, nullptr, r0, B, Bp, s->F, s->T, s->stdv, s->stdv + kMlpPad,
        s->stdv + 2 * kMlpPad, s->stdv + 3 * kMlpPad, s->X, nullptr);
    mlp_infer(s, s->X, Bp, s->P, st);
    unstd_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(
        s->P, B, s->T, s->q, s->stdv + 2 * kMlpPad, s->stdv + 3 * kMlpPad, out + r0 * s->T);
  }
  rc = launch_check();
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = CFUST_EHIP;
  return rc;
}

int cfust_surrogate_get_state(const cfust_surrogate* s, float* params, float* stdv) {
  if (!s) return CFUST_EINVAL;
  if (params && hipMemcpy(params, s->params, kMlpParams * sizeof(float), hipMemcpyDeviceToHost) !=
                    hipSuccess)
    return CFUST_EHIP;
  if (stdv) memcpy(stdv, s->h_std, sizeof(s->h_std));
  return CFUST_OK;
}

int cfust_surrogate_set_state(cfust_surrogate* s, const float* params, const float* stdv) {
  if (!s) return CFUST_EINVAL;
  if (params) {
    if (hipMemcpy(s->params, params, kMlpParams * sizeof(float), hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemset(s->adm, 0, kMlpParams * sizeof(float)) != hipSuccess ||
        hipMemset(s->adv, 0, kMlpParams * sizeof(float)) != hipSuccess)
      return CFUST_EHIP;
    s->adam_t = 0;
    int rc = refresh_bf16(s, nullptr);
    if (rc) return rc;
  }
  if (stdv) {
    for (int c = 0; c < CFUST_SURR_STD; ++c)
      if (!std::isfinite(stdv[c]) || ((c / kMlpPad) % 2 == 1 && !(stdv[c] > 0.f)))
        return CFUST_EINVAL;
    memcpy(s->h_std, stdv, sizeof(s->h_std));
    if (hipMemcpy(s->stdv, s->h_std, sizeof(s->h_std), hipMemcpyHostToDevice) != hipSuccess)
      return CFUST_EHIP;
    s->have_std = true;
  }
  return hipDeviceSynchronize() == hipSuccess ? CFUST_OK : CFUST_EHIP;
}

int cfust_surrogate_save(const cfust_surrogate* s, const char* path) {
  if (!s || !path) return CFUST_EINVAL;
  std::vector<float> w((size_t)kMlpParams);
  int rc = cfust_surrogate_get_state(s, w.data(), nullptr);
  if (rc) return rc;
  SurrFileHeader hd{};
  memcpy(hd.magic, "CFUSTNN1", 8);
  hd.version = 1;
  hd.q = s->q;
  hd.F = s->F;
  hd.T = s->T;
  hd.hidden = kMlpHid;
  hd.layers = kMlpLayers;
  hd.nparams = kMlpParams;
  const SurrRange& r = s->rg;
  const double rr[6] = {r.h_lo, r.h_hi, r.dof_lo, r.dof_hi, r.r_max, r.eig_min};
  memcpy(hd.range, rr, sizeof(rr));
  FILE* f = fopen(path, "wb");
  if (!f) return CFUST_EINVAL;
  bool ok = fwrite(&hd, sizeof(hd), 1, f) == 1 &&
            fwrite(s->h_std, sizeof(float), CFUST_SURR_STD, f) == (size_t)CFUST_SURR_STD &&
            fwrite(w.data(), sizeof(float), w.size(), f) == w.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? CFUST_OK : CFUST_EINVAL;
}

int cfust_surrogate_load(const char* path, cfust_surrogate** out) {
  if (!path || !out) return CFUST_EINVAL;
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return CFUST_EINVAL;
  SurrFileHeader hd{};
  std::vector<float> stdv(CFUST_SURR_STD), w((size_t)kMlpParams);
  bool ok = fread(&hd, sizeof(hd), 1, f) == 1 && memcmp(hd.magic, "CFUSTNN1", 8) == 0 &&
            hd.version == 1 && hd.q >= 1 && hd.q <= kMaxQFull && hd.F == surr_feat_width(hd.q) &&
            hd.T == surr_targ_width(hd.q) && hd.hidden == kMlpHid && hd.layers == kMlpLayers &&
            hd.nparams == kMlpParams &&
            fread(stdv.data(), sizeof(float), CFUST_SURR_STD, f) == (size_t)CFUST_SURR_STD &&
            fread(w.data(), sizeof(float), w.size(), f) == w.size();
  fclose(f);
  if (!ok) return CFUST_EINVAL;
  cfust_surrogate* s = nullptr;
  int rc = cfust_surrogate_create(hd.q, hd.range, 0, &s);
  if (rc) return rc;
  if ((rc = cfust_surrogate_set_state(s, w.data(), stdv.data()))) {
    cfust_surrogate_destroy(s);
    return rc;
  }
  *out = s;
  return CFUST_OK;
}

int64_t cfust_surrogate_fallback_count(const cfust_surrogate* s) {
  if (!s) return -1;
  unsigned long long v = 0;
  if (hipMemcpy(&v, s->fb_total, sizeof(v), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return (int64_t)v;
}

int cfust_surrogate_em_switch(const cfust_surrogate* s) { return s ? s->em_switch : -1; }

int cfust_surrogate_adapt(cfust_surrogate* s, const double* y, int64_t n, int p, int q, int g,
                          const double* pi, const double* mu, const double* Sigma,
                          const double* Delta, const double* nu, const double* u, int n_qmc,
                          int64_t samples, int epochs, unsigned long long seed,
                          const cfust_opts* o, double* loss, int64_t* rows) {
  if (loss) *loss = 0.0;
  if (rows) *rows = 0;
  int rc = check_dims(n, p, q, g, n_qmc);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if (!s || !y || !pi || !mu || !Sigma || !Delta || !nu || !u || n < 1 || samples < 1 ||
      epochs < 0 || s->q != q || !s->have_std)
    return CFUST_EINVAL;
  cfust_opts oo;
  cfust_default_opts(&oo);
  oo.stream = o ? o->stream : nullptr;
  Plan pl = make_plan(0, p, q, g, 1, CFUST_FP64);
  Ws ws;
  if ((rc = acquire(pl, &oo, &ws))) return rc;
  hipStream_t st = ws.st;
  clear_status(ws, pl);
  const double* comp = ws.at<double>(pl.o_comp);
  int* status = ws.at<int>(pl.o_status);
  precompute_kernel<<<1, kPrecompThreads, precompute_lds_bytes(p, q, g), st>>>(
      p, q, g, pi, Sigma, Delta, mu, nu,
                                      ws.at<double>(pl.o_comp), status);
  // uniform sample of pairs (with replacement)
  const int64_t pairs = n * g;
  const int F = s->F, T = s->T;
  std::vector<int64_t> pick((size_t)samples);
  Rng rng{seed * 0x9E3779B97F4A7C15ull + 0x5851F42D4C957F2Dull};
  for (auto& k : pick) k = (int64_t)(rng.next() % (uint64_t)pairs);
  int64_t* pick_d = nullptr;
  double* feat_d = nullptr;
  if (hipMallocAsync((void**)&pick_d, samples * sizeof(int64_t), st) != hipSuccess ||
      hipMallocAsync((void**)&feat_d, (size_t)2 * samples * F * sizeof(double), st) !=
          hipSuccess) {
    if (pick_d) (void)hipFreeAsync(pick_d, st);
    release(&ws);
    return CFUST_ENOMEM;
  }
  (void)hipMemcpyAsync(pick_d, pick.data(), samples * sizeof(int64_t), hipMemcpyHostToDevice, st);
  const unsigned nb = (unsigned)((samples + 127) / 128);
  if (p <= 8)
    launch_features_list<8>(q, nb, st, y, p, g, mu, comp, pick_d, samples, feat_d, status);
  else
    launch_features_list<kMaxP>(q, nb, st, y, p, g, mu, comp, pick_d, samples, feat_d, status);
  std::vector<double> fh((size_t)2 * samples * F);
  rc = launch_check();
  if (!rc && hipMemcpyAsync(fh.data(), feat_d, fh.size() * sizeof(double), hipMemcpyDeviceToHost,
                            st) != hipSuccess)
    rc = CFUST_EHIP;
  if (!rc) rc = fetch_status(ws, pl, nullptr);
  (void)hipFreeAsync(pick_d, st);
  (void)hipFreeAsync(feat_d, st);
  if (rc) {
    release(&ws);
    return rc;
  }
  // rows inside the training range
  const SurrRange& r = s->rg;
  std::vector<double> hs, Rs, dofs, fs;
  for (int64_t k = 0; k < 2 * samples; ++k) {
    double* f = fh.data() + k * F;
    bool in = f[F - 1] >= r.dof_lo && f[F - 1] <= r.dof_hi;
    // as in the E-step: bounds above h_hi lowered to h_hi, below h_lo out
    for (int a = 0; a < q; ++a) f[a] = fmin(f[a], r.h_hi);
    for (int a = 0; a < q && in; ++a) in = f[a] >= r.h_lo;
    for (int a = q; a < F - 1 && in; ++a) in = fabs(f[a]) <= r.r_max;
    if (!in) continue;
    fs.insert(fs.end(), f, f + F);
    hs.insert(hs.end(), f, f + q);
    dofs.push_back(f[F - 1]);
    const size_t b = Rs.size();
    Rs.resize(b + (size_t)q * q);
    int t = q;
    for (int a = 0; a < q; ++a) {
      Rs[b + a * q + a] = 1.0;
      for (int c = a + 1; c < q; ++c, ++t) {
        Rs[b + a * q + c] = f[t];
        Rs[b + c * q + a] = f[t];
      }
    }
  }
  const int64_t M = (int64_t)dofs.size();
  if (rows) *rows = M;
  if (M == 0 || epochs == 0) {
    release(&ws);
    return CFUST_OK;
  }
  double *h_d = nullptr, *R_d = nullptr, *dof_d = nullptr, *f_d = nullptr, *lab_d = nullptr;
  bool ok = hipMallocAsync((void**)&h_d, hs.size() * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&R_d, Rs.size() * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&dof_d, dofs.size() * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&f_d, fs.size() * sizeof(double), st) == hipSuccess &&
            hipMallocAsync((void**)&lab_d, (size_t)M * T * sizeof(double), st) == hipSuccess;
  if (ok) {
    (void)hipMemcpyAsync(h_d, hs.data(), hs.size() * sizeof(double), hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(R_d, Rs.data(), Rs.size() * sizeof(double), hipMemcpyHostToDevice, st);
    (void)hipMemcpyAsync(dof_d, dofs.data(), dofs.size() * sizeof(double), hipMemcpyHostToDevice,
                         st);
    (void)hipMemcpyAsync(f_d, fs.data(), fs.size() * sizeof(double), hipMemcpyHostToDevice, st);
    rc = run_ghk_batch<double>(q, M, h_d, R_d, dof_d, u, n_qmc, lab_d, st);
    if (!rc) {
      std::vector<float> wo((size_t)T, 1.0f);
      wo[0] = (float)(T - 1);
      std::vector<double> trace((size_t)epochs);
      rc = cfust_surrogate_train(s, f_d, lab_d, M, epochs, 1024, 5e-4, 1e-6, seed, wo.data(), &oo,
                                 trace.data());
      if (!rc && loss) *loss = trace[epochs - 1];
    }
  } else {
    rc = CFUST_ENOMEM;
  }
  for (double* ptr : {h_d, R_d, dof_d, f_d, lab_d})
    if (ptr) (void)hipFreeAsync(ptr, st);
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = CFUST_EHIP;
  release(&ws);
  return rc;
}

int cfust_pair_features(const double* y, int64_t n, int p, int q, int g, const double* pi,
                        const double* mu, const double* Sigma, const double* Delta,
                        const double* nu, const cfust_opts* o, double* out) {
  int rc = check_dims(n, p, q, g, 1);
  if (rc) return rc;
  if ((rc = check_opts(o))) return rc;
  if (q > kMaxQFull) return CFUST_EINVAL;
  if ((n > 0 && (!y || !out)) || !pi || !mu || !Sigma || !Delta || !nu) return CFUST_EINVAL;
  Plan pl = make_plan(0, p, q, g, 1, CFUST_FP64);
  Ws ws;
  cfust_opts oo;
  cfust_default_opts(&oo);
  oo.stream = o ? o->stream : nullptr;
  if ((rc = acquire(pl, &oo, &ws))) return rc;
  clear_status(ws, pl);
  const double* comp = ws.at<double>(pl.o_comp);
  int* status = ws.at<int>(pl.o_status);
  precompute_kernel<<<1, kPrecompThreads, precompute_lds_bytes(p, q, g), ws.st>>>(
      p, q, g, pi, Sigma, Delta, mu, nu,
                                         ws.at<double>(pl.o_comp), status);
  const int64_t pairs = n * g;
  const unsigned nb = (unsigned)((pairs + 127) / 128);
  if (pairs > 0) {
    if (p <= 8)
      launch_pair_features<8>(q, nb, ws.st, y, n, p, g, mu, comp, out, status);
    else
      launch_pair_features<kMaxP>(q, nb, ws.st, y, n, p, g, mu, comp, out, status);
  }
  rc = launch_check();
  int stt = fetch_status(ws, pl, nullptr);
  release(&ws);
  return rc ? rc : stt;
}

int cfust_mlp_gemm(int ta, int tb, int M, int N, int K, const unsigned short* A,
                   const unsigned short* B, float* C, void* stream) {
  if (M < 64 || N < 64 || K < 32 || M % 64 || N % 64 || K % 32 || !A || !B || !C)
    return CFUST_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  Epi ep{};
  ep.C = C;
  ep.ldc = N;
  const int lda = ta ? M : K, ldb = tb ? K : N;
  if (!ta && !tb) gemm<false, false, kEpiStore>(A, nullptr, lda, B, ldb, M, N, K, 1, ep, st);
  if (!ta && tb) gemm<false, true, kEpiStore>(A, nullptr, lda, B, ldb, M, N, K, 1, ep, st);
  if (ta && !tb) gemm<true, false, kEpiStore>(A, nullptr, lda, B, ldb, M, N, K, 1, ep, st);
  if (ta && tb) gemm<true, true, kEpiStore>(A, nullptr, lda, B, ldb, M, N, K, 1, ep, st);
  int rc = launch_check();
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = CFUST_EHIP;
  return rc;
}

}  // extern "C"
