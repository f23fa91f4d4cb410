// Host-side pieces shared by the translation units of the library: the
// workspace plan of one E-step / M-step call, the per-call launch context,
// argument checks and the launchers each unit exports to the others.
//
//   cfust_capi.hip        the C ABI of the single-problem EM (E-step, M-step,
//                         log-likelihood, EM driver with Aitken's rule) and
//                         the shared helpers declared here
//   cfust_pairs_*.hip     the pair-kernel launchers of one integrand type
//                         and a range of q (the long compiles, built in
//                         parallel)
//   cfust_batched.hip     the batched form, its autotuner and graph replay,
//                         multistart (Algorithm 1) and the randomised-QMC
//                         error bar
//   cfust_surrogate.hip   the surrogate network handle, training, inference,
//                         adaptation, GHK label batches
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/cfust.h"

namespace cfust {
namespace host {

// Workspace plan of one call: sizes and byte offsets inside the workspace.
struct Plan {
  int64_t n;
  int p, q, g, N, prec;
  int W, S, GS, stride;
  int tile, nb, ny;
  int64_t per_block;
  size_t lds_bytes;
  bool exact = false;    // exact E[log W | y] (nu_mode EXACT)
  bool reorder = false;  // Genz-Bretz variable order per pair (opts.reorder)
  // byte offsets inside the workspace
  size_t o_tA;  // tangent of integral A's chi scale (exact E[log W | y])
  size_t o_status, o_comp, o_uT, o_ubT, o_sA, o_sB, o_rsB, o_pair, o_part, o_pll, o_pitmp, o_mwork,
      o_ll, o_stats, total;
  // waves per pair (pair_part_kernel + pair_finish_kernel when > 1)
  int split = 1;
  size_t o_parts = 0;
  // surrogate check (difference estimator over m sampled observations)
  int64_t check_m = 0;
  int64_t chk_per_block = 0;
  int chk_nb = 0;
  size_t o_chk_y = 0, o_chk_rnet = 0, o_chk_rghk = 0, o_chk_part = 0, o_chk_pll = 0,
         o_chk_stats = 0;
};

// Launch context of one call: workspace base, stream, optional timing
// events and the surrogate network.
struct Ws {
  char* base = nullptr;
  bool owned = false;
  hipStream_t st = nullptr;
  double* prof = nullptr;           // host accumulator, CFUST_PROF_SLOTS entries
  cfust_surrogate* surr = nullptr;  // surrogate network for the pair integrals
  hipEvent_t ev[2 * CFUST_PROF_SLOTS] = {};
  bool ev_pending[CFUST_PROF_SLOTS] = {};
  template <typename X>
  X* at(size_t off) const {
    return reinterpret_cast<X*>(base + off);
  }
};

// ---- cfust_capi.hip ----
size_t align_up(size_t x);
Plan make_plan(int64_t n, int p, int q, int g, int N, int prec, int64_t check_m = 0);
int check_dims(int64_t n, int p, int q, int g, int N);
int check_opts(const cfust_opts* o);
int acquire(const Plan& pl, const cfust_opts* o, Ws* ws);
void release(Ws* ws);
int launch_check();
void clear_status(const Ws& ws, const Plan& pl);
int fetch_status(Ws& ws, const Plan& pl, int* bad);
// the per-component blocks of g components (pi, mu, Sigma, Delta, nu)
void launch_precompute(const Ws& ws, const Plan& pl, const double* pi, const double* mu,
                       const double* Sigma, const double* Delta, const double* nu);

// ---- cfust_pairs_*.hip: the pair kernels of one q ----
template <typename T, int Q, bool MOM>
void launch_pairs_q(const Ws& ws, const Plan& pl, const double* y, const double* mu);

// ---- cfust_surrogate.hip ----
// E-step pairs through the network, out-of-range pairs through the GHK kernel
template <typename T>
int launch_surrogate_pairs(const Ws& ws, const Plan& pl, const double* y, const double* mu);
// the handle holds a trained network for this q
bool surrogate_ready(const cfust_surrogate* s, int q);
// records the first GHK E-step of a two-phase fit (-1: none yet)
void surrogate_set_switch(cfust_surrogate* s, int t);

}  // namespace host
}  // namespace cfust
