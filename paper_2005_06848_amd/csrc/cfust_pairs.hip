// Pair-kernel launchers of one E-step (section 3.2, Algorithm 2): the GHK
// integrals of every (observation, component) pair, one wave per pair or a
// pair split over several waves.  This file is compiled once per integrand
// type and range of q (CFUST_PAIRS_T, CFUST_PAIRS_QLO..CFUST_PAIRS_QHI), so
// that the long compiles of the fully unrolled kernels run in parallel.
#include <hip/hip_runtime.h>

#include "cfust_host.hpp"
#include "cfust_kernels.hpp"

#ifndef CFUST_PAIRS_T
#error "CFUST_PAIRS_T (double or float) and the q range must be defined"
#endif

using namespace cfust;

namespace cfust {
namespace host {

template <typename T, int Q, bool MOM>
void launch_pairs_q(const Ws& ws, const Plan& pl, const double* y, const double* mu) {
  int64_t pairs = pl.n * pl.g;
  if (pairs == 0) return;
  unsigned blocks = (unsigned)((pairs + 3) / 4);
  // Resident waves per SIMD asked of the compiler.  FP64 q <= 4: four (2.5%
  // faster at p=q=4, 48 B/lane of spill outside the point loop).  FP64
  // q = 5, 6: three (3.8% faster at p=q=6 than the compiler's two, despite
  // 192 B/lane of spill).  FP32 q = 5: four (7.6% faster than the
  // compiler's choice at p=q=5).  FP32 q = 6 and larger q keep the
  // compiler's choice (at p=q=6 four waves spill 176 B/lane and are 8%
  // slower).
  constexpr int OCC = (sizeof(T) == 8 && Q <= 4)        ? 4
                      : (sizeof(T) == 8 && (Q == 5 || Q == 6)) ? 3
                      : (sizeof(T) == 4 && Q == 5)             ? 4
                                                               : 0;
  const double* comp = ws.at<double>(pl.o_comp);
  double* pairs_out = ws.at<double>(pl.o_pair);
  int* status = ws.at<int>(pl.o_status);
  const T *sA = ws.at<T>(pl.o_sA), *sB = ws.at<T>(pl.o_sB), *rsB = ws.at<T>(pl.o_rsB);
  const T *uT = ws.at<T>(pl.o_uT), *ubT = ws.at<T>(pl.o_ubT);
  const T* tA = pl.exact ? ws.at<T>(pl.o_tA) : nullptr;
  // The exact-nu variants (tangent of integral A) exist for the E-step only
  // (MOM) and keep the compiler's occupancy in the one-wave kernel, as do the
  // ordered ones (both add registers).  Above kMaxQFull the ordered kernels
  // do not exist (the entry points reject the ordering there).
  if (pl.split > 1 && !pl.reorder) {
    const int K = pl.split;
    double* parts = ws.at<double>(pl.o_parts);
    const unsigned pblocks = (unsigned)((pairs * K + 3) / 4);
    if constexpr (MOM) {
      if (pl.exact) {
        pair_part_kernel<T, Q, MOM, OCC, true><<<pblocks, 256, 0, ws.st>>>(
            y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, K, parts, status, tA);
        pair_finish_kernel<T, Q, MOM, true><<<blocks, 256, 0, ws.st>>>(
            y, pl.n, pl.p, pl.g, mu, comp, pl.N, K, parts, pairs_out, pl.W, status);
        return;
      }
    }
    pair_part_kernel<T, Q, MOM, OCC><<<pblocks, 256, 0, ws.st>>>(
        y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, K, parts, status);
    pair_finish_kernel<T, Q, MOM><<<blocks, 256, 0, ws.st>>>(
        y, pl.n, pl.p, pl.g, mu, comp, pl.N, K, parts, pairs_out, pl.W, status);
    return;
  }
  if constexpr (MOM) {
    if (pl.exact) {
      if constexpr (Q <= kMaxQFull) {
        if (pl.reorder) {
          pair_kernel<T, Q, MOM, 0, true, true><<<blocks, 256, 0, ws.st>>>(
              y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, pairs_out, pl.W, status,
              tA);
          return;
        }
      }
      pair_kernel<T, Q, MOM, 0, true><<<blocks, 256, 0, ws.st>>>(
          y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, pairs_out, pl.W, status, tA);
      return;
    }
  }
  if constexpr (Q <= kMaxQFull) {
    if (pl.reorder) {
      pair_kernel<T, Q, MOM, 0, false, true><<<blocks, 256, 0, ws.st>>>(
          y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, pairs_out, pl.W, status);
      return;
    }
  }
  // natural order
  pair_kernel<T, Q, MOM, OCC><<<blocks, 256, 0, ws.st>>>(
      y, pl.n, pl.p, pl.g, mu, comp, sA, sB, rsB, uT, ubT, pl.N, pairs_out, pl.W, status);
}


#define CFUST_PAIRS_INST(Q)                                                                  \
  template void launch_pairs_q<CFUST_PAIRS_T, Q, true>(const Ws&, const Plan&, const double*, \
                                                       const double*);                        \
  template void launch_pairs_q<CFUST_PAIRS_T, Q, false>(const Ws&, const Plan&, const double*, \
                                                        const double*);
#if CFUST_PAIRS_QLO <= 1 && 1 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(1)
#endif
#if CFUST_PAIRS_QLO <= 2 && 2 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(2)
#endif
#if CFUST_PAIRS_QLO <= 3 && 3 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(3)
#endif
#if CFUST_PAIRS_QLO <= 4 && 4 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(4)
#endif
#if CFUST_PAIRS_QLO <= 5 && 5 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(5)
#endif
#if CFUST_PAIRS_QLO <= 6 && 6 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(6)
#endif
#if CFUST_PAIRS_QLO <= 7 && 7 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(7)
#endif
#if CFUST_PAIRS_QLO <= 8 && 8 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(8)
#endif
#if CFUST_PAIRS_QLO <= 9 && 9 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(9)
#endif
#if CFUST_PAIRS_QLO <= 10 && 10 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(10)
#endif
#if CFUST_PAIRS_QLO <= 11 && 11 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(11)
#endif
#if CFUST_PAIRS_QLO <= 12 && 12 <= CFUST_PAIRS_QHI
CFUST_PAIRS_INST(12)
#endif

}  // namespace host
}  // namespace cfust
