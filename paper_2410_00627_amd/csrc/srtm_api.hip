// C-ABI entry points: argument validation, workspace sizing and kernel dispatch.
// Nothing here allocates memory or synchronises; argument errors return before any
// HIP call is made.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "srtm_layout.h"
#include "../../include/srtm.h"

namespace srtm {
struct Ptrs {
  const void *F, *Q, *H, *R, *m0, *P0, *y;
  void *ms_fast, *Ps_fast, *ms_slow, *Ps_slow;
  void *mf_fast, *Pf_fast, *mf_slow, *Pf_slow;
  void* ws;
  int32_t* info;
};
bool pair_supported(int nx, int ny);
srtm_status dispatch(const srtm_shape& sh, const Ptrs& p, bool smoother, hipStream_t st, hipEvent_t const* ev,
                     int nev);
size_t constants_lds_bytes(int nx, int ny, int L);
}  // namespace srtm

namespace {

constexpr size_t kMaxLds = 160 * 1024;

bool aligned(const void* p, uintptr_t a) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) % a) == 0; }

srtm_status check_shape(const srtm_shape* sh) {
  if (!sh) return SRTM_E_NULL;
  if (sh->dtype != SRTM_F32 && sh->dtype != SRTM_F64) return SRTM_E_DTYPE;
  if (sh->nx < 1 || sh->ny < 1 || sh->L < 1 || sh->N < 1) return SRTM_E_SHAPE;
  if (!srtm::pair_supported(sh->nx, sh->ny)) return SRTM_E_UNSUPPORTED;
  if (sh->L > SRTM_MAX_L || sh->N > SRTM_MAX_N) return SRTM_E_UNSUPPORTED;
  if (srtm::constants_lds_bytes(sh->nx, sh->ny, sh->L) > kMaxLds) return SRTM_E_UNSUPPORTED;
  return SRTM_OK;
}

srtm_status run_common(const srtm_shape* sh, const srtm::Ptrs& p, bool smoother, size_t ws_bytes, void* stream,
                       void* const* events, int32_t n_events) {
  srtm_status s = check_shape(sh);
  if (s != SRTM_OK) return s;
  if (!p.F || !p.Q || !p.H || !p.R || !p.m0 || !p.P0 || !p.y || !p.ws) return SRTM_E_NULL;
  const void* all[] = {p.F, p.Q, p.H, p.R, p.m0, p.P0, p.y, p.ms_fast, p.Ps_fast, p.ms_slow,
                       p.Ps_slow, p.mf_fast, p.Pf_fast, p.mf_slow, p.Pf_slow};
  for (const void* q : all)
    if (!aligned(q, 16)) return SRTM_E_ALIGN;
  if (!aligned(p.ws, 256) || !aligned(p.info, 4)) return SRTM_E_ALIGN;
  const size_t esz = sh->dtype == SRTM_F64 ? 8 : 4;
  const srtm::WorkLayout wl = srtm::make_work_layout(sh->nx, sh->ny, sh->L, sh->N, esz, smoother);
  if (ws_bytes < wl.total) return SRTM_E_WORKSPACE;
  if (events && n_events < 2 * srtm_kernel_count(smoother ? 1 : 0)) return SRTM_E_SHAPE;
  return srtm::dispatch(*sh, p, smoother, static_cast<hipStream_t>(stream),
                        reinterpret_cast<hipEvent_t const*>(events), events ? n_events : 0);
}

const char* const kFilterKernels[] = {"k_constants", "k_fwd_reduce", "k_fwd_tiles", "k_fwd_final", "k_recover"};
const char* const kSmoothKernels[] = {"k_constants", "k_fwd_reduce", "k_fwd_tiles",
                                      "k_fwd_bwd",   "k_bwd_tiles",  "k_recover"};

}  // namespace

extern "C" {

srtm_status srtm_workspace_size(const srtm_shape* shape, int32_t smoother, size_t* bytes) {
  srtm_status s = check_shape(shape);
  if (s != SRTM_OK) return s;
  if (!bytes) return SRTM_E_NULL;
  const size_t esz = shape->dtype == SRTM_F64 ? 8 : 4;
  *bytes = srtm::make_work_layout(shape->nx, shape->ny, shape->L, shape->N, esz, smoother != 0).total;
  return SRTM_OK;
}

int32_t srtm_supported(int32_t nx, int32_t ny) { return srtm::pair_supported(nx, ny) ? 1 : 0; }

srtm_status srtm_filter(const srtm_shape* shape, const void* F, const void* Q, const void* H, const void* R,
                        const void* m0, const void* P0, const void* y, void* m_fast, void* P_fast, void* m_slow,
                        void* P_slow, void* workspace, size_t workspace_bytes, int32_t* info, void* stream) {
  const srtm::Ptrs p{F, Q, H, R, m0, P0, y, nullptr, nullptr, nullptr, nullptr,
                     m_fast, P_fast, m_slow, P_slow, workspace, info};
  return run_common(shape, p, false, workspace_bytes, stream, nullptr, 0);
}

srtm_status srtm_smooth(const srtm_shape* shape, const void* F, const void* Q, const void* H, const void* R,
                        const void* m0, const void* P0, const void* y, void* ms_fast, void* Ps_fast,
                        void* ms_slow, void* Ps_slow, void* mf_fast, void* Pf_fast, void* mf_slow,
                        void* Pf_slow, void* workspace, size_t workspace_bytes, int32_t* info, void* stream) {
  const srtm::Ptrs p{F, Q, H, R, m0, P0, y, ms_fast, Ps_fast, ms_slow, Ps_slow,
                     mf_fast, Pf_fast, mf_slow, Pf_slow, workspace, info};
  return run_common(shape, p, true, workspace_bytes, stream, nullptr, 0);
}

srtm_status srtm_smooth_profiled(const srtm_shape* shape, const void* F, const void* Q, const void* H,
                                 const void* R, const void* m0, const void* P0, const void* y, void* ms_fast,
                                 void* Ps_fast, void* ms_slow, void* Ps_slow, void* mf_fast, void* Pf_fast,
                                 void* mf_slow, void* Pf_slow, void* workspace, size_t workspace_bytes,
                                 int32_t* info, void* stream, void* const* events, int32_t n_events) {
  if (!events) return SRTM_E_NULL;
  const srtm::Ptrs p{F, Q, H, R, m0, P0, y, ms_fast, Ps_fast, ms_slow, Ps_slow,
                     mf_fast, Pf_fast, mf_slow, Pf_slow, workspace, info};
  return run_common(shape, p, true, workspace_bytes, stream, events, n_events);
}

int32_t srtm_kernel_count(int32_t smoother) {
  return smoother ? (int32_t)(sizeof(kSmoothKernels) / sizeof(kSmoothKernels[0]))
                  : (int32_t)(sizeof(kFilterKernels) / sizeof(kFilterKernels[0]));
}

const char* srtm_kernel_name(int32_t smoother, int32_t j) {
  if (j < 0 || j >= srtm_kernel_count(smoother)) return nullptr;
  return smoother ? kSmoothKernels[j] : kFilterKernels[j];
}

const char* srtm_status_string(int32_t status) {
  switch (status) {
    case SRTM_OK: return "ok";
    case SRTM_E_NULL: return "a required pointer is NULL";
    case SRTM_E_SHAPE: return "invalid shape (N, L, nx, ny must be >= 1) or event count";
    case SRTM_E_DTYPE: return "dtype must be SRTM_F32 or SRTM_F64";
    case SRTM_E_UNSUPPORTED: return "unsupported (nx, ny) pair, or L / N above this build's limits";
    case SRTM_E_ALIGN: return "array not 16-byte aligned (workspace: 256 bytes)";
    case SRTM_E_WORKSPACE: return "workspace smaller than srtm_workspace_size()";
    case SRTM_E_HIP: return "HIP runtime error while enqueueing work";
    default: return "unknown status";
  }
}

int32_t srtm_version(void) { return 100; }

}  // extern "C"
