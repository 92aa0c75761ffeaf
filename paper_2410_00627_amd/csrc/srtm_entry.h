// Host-side interface between the C-ABI code (srtm_api.hip) and the kernel translation units.
// srtm_kernels.hip is compiled once per supported (nx, ny) pair (-DSRTM_NX, -DSRTM_NY); each
// object defines that pair's run_pair_<nx>_<ny> and run_batch_pair_<nx>_<ny>. It is compiled
// once more per element type (-DSRTM_MIXED_T=float / double) for the mixed-pair batches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/srtm.h"

// The (nx, ny) pairs compiled into the library.
#define SRTM_PAIRS(X) X(1, 1) X(2, 1) X(2, 2) X(3, 1) X(3, 2) X(4, 1) X(4, 2) X(6, 1)

namespace srtm {

// Device pointers of one single-sequence call (outputs nullable). With known inputs, B [nx][nu]
// and u [N][L][nu] are set and nu >= 1; without, both are null and nu = 0.
struct Ptrs {
  const void *F, *Q, *H, *R, *m0, *P0, *y;
  void *ms_fast, *Ps_fast, *ms_slow, *Ps_slow;
  void *mf_fast, *Pf_fast, *mf_slow, *Pf_slow;
  void* ws;
  int32_t* info;
  const void* B = nullptr;
  const void* u = nullptr;
  int nu = 0;
  bool tv = false;  // F, Q, H, R given per window ([N][...]); no inputs then
  void* Cs_fast = nullptr;  // lag-one smoothed cross-covariances [N][L][nx][nx] (srtm_smooth_lag1)
};

// Largest state size of the per-window (time-varying) path: its scans hold whole filter
// elements of all 256 windows of a tile in LDS.
constexpr int TV_NX_MAX = 4;

// What follows the scans: fast-rate recovery modes 1 (filter), 2 (smoother), 3 (both), the
// log-likelihood alone (REC_LL) or the log-likelihood and its gradient (REC_GRAD). REC_SEQ
// selects the sequential comparator instead of the scans (srtm_smooth_sequential).
constexpr int REC_LL = 4, REC_GRAD = 5, REC_SEQ = 6;

// Largest input size of the kernels with known inputs.
constexpr int NU_MAX = SRTM_MAX_NU;

#define SRTM_PAIR_DECL(a, b)                                                                                      \
  srtm_status run_pair_##a##_##b(int dtype, const srtm_shape& sh, const Ptrs& p, bool smoother, hipStream_t st,  \
                                 hipEvent_t const* ev, int nev, int lik_mode, void* ll, void* dF, void* dQ,       \
                                 void* dR);                                                                       \
  srtm_status run_batch_pair_##a##_##b(int dtype, const void* table, int nseq, int64_t ntiles, int max_L,        \
                                       void* ws, int32_t* info, hipStream_t st, bool grad);
SRTM_PAIRS(SRTM_PAIR_DECL)
#undef SRTM_PAIR_DECL

struct SeqDesc;
// Mixed-pair batches (srtm_smooth_batch_ex): one object per element type. `host` is the host
// copy of the validated table, `table_dev` its device copy.
srtm_status run_mixed_double(const SeqDesc* host, const void* table_dev, int nseq, int64_t ntiles, int max_L,
                             void* ws, int32_t* info, hipStream_t st);
srtm_status run_mixed_float(const SeqDesc* host, const void* table_dev, int nseq, int64_t ntiles, int max_L,
                            void* ws, int32_t* info, hipStream_t st);

}  // namespace srtm
