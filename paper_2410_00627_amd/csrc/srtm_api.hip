// C-ABI entry points: argument validation, workspace sizing and kernel dispatch.
// Nothing here allocates memory or synchronises; argument errors return before any
// HIP call is made.

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "srtm_entry.h"
#include "srtm_layout.h"

// Workspace of srtm_smooth_noalloc: one array per GPU, resident until the process ends. Host
// code never passes `scratch` itself to a kernel (on the host it only names the symbol); it
// uses the device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[SRTM_NOALLOC_SCRATCH_BYTES];

namespace srtm {
bool pair_supported(int nx, int ny) {
#define SRTM_SUP(a, b) \
  if (nx == a && ny == b) return true;
  SRTM_PAIRS(SRTM_SUP)
#undef SRTM_SUP
  return false;
}

// Routes a call to the object compiled for its (nx, ny) pair (lik_mode: 0, REC_LL or REC_GRAD).
srtm_status dispatch(const srtm_shape& sh, const Ptrs& p, bool smoother, hipStream_t st, hipEvent_t const* ev,
                     int nev, int lik_mode = 0, void* ll = nullptr, void* dF = nullptr, void* dQ = nullptr,
                     void* dR = nullptr) {
#define SRTM_DISP(a, b) \
  if (sh.nx == a && sh.ny == b) return run_pair_##a##_##b(sh.dtype, sh, p, smoother, st, ev, nev, lik_mode, ll, dF, dQ, dR);
  SRTM_PAIRS(SRTM_DISP)
#undef SRTM_DISP
  return SRTM_E_UNSUPPORTED;
}

srtm_status dispatch_batch(int nx, int ny, int dtype, const void* table, int nseq, int64_t ntiles, int max_L,
                           void* ws, int32_t* info, hipStream_t st, bool grad) {
#define SRTM_DISPB(a, b) \
  if (nx == a && ny == b) return run_batch_pair_##a##_##b(dtype, table, nseq, ntiles, max_L, ws, info, st, grad);
  SRTM_PAIRS(SRTM_DISPB)
#undef SRTM_DISPB
  return SRTM_E_UNSUPPORTED;
}
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
                       p.Ps_slow, p.mf_fast, p.Pf_fast, p.mf_slow, p.Pf_slow, p.Cs_fast};
  for (const void* q : all)
    if (!aligned(q, 16)) return SRTM_E_ALIGN;
  if (!aligned(p.ws, 256) || !aligned(p.info, 4)) return SRTM_E_ALIGN;
  const size_t esz = sh->dtype == SRTM_F64 ? 8 : 4;
  if (p.tv && sh->nx > srtm::TV_NX_MAX) return SRTM_E_UNSUPPORTED;
  const srtm::WorkLayout wl =
      srtm::make_work_layout(sh->nx, sh->ny, sh->L, sh->N, esz, smoother, p.B != nullptr, p.tv);
  if (ws_bytes < wl.total) return SRTM_E_WORKSPACE;
  if (events && n_events < 2 * srtm_kernel_count(smoother ? 1 : 0)) return SRTM_E_SHAPE;
  return srtm::dispatch(*sh, p, smoother, static_cast<hipStream_t>(stream),
                        reinterpret_cast<hipEvent_t const*>(events), events ? n_events : 0);
}

// Adds validated known inputs to `p`.
srtm_status with_inputs(const srtm_inputs* in, srtm::Ptrs& p) {
  if (!in || !in->B || !in->u) return SRTM_E_NULL;
  if (in->nu < 1 || in->nu > SRTM_MAX_NU || in->reserved != 0) return SRTM_E_SHAPE;
  if (!aligned(in->B, 16) || !aligned(in->u, 16)) return SRTM_E_ALIGN;
  p.B = in->B;
  p.u = in->u;
  p.nu = in->nu;
  return SRTM_OK;
}

// Device address of `scratch` on the current device, looked up once per device (with that
// device current) and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

srtm_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SRTM_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return SRTM_E_HIP;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return SRTM_OK;
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

srtm_status srtm_workspace_size_inputs(const srtm_shape* shape, int32_t smoother, size_t* bytes) {
  srtm_status s = check_shape(shape);
  if (s != SRTM_OK) return s;
  if (!bytes) return SRTM_E_NULL;
  const size_t esz = shape->dtype == SRTM_F64 ? 8 : 4;
  *bytes = srtm::make_work_layout(shape->nx, shape->ny, shape->L, shape->N, esz, smoother != 0, true).total;
  return SRTM_OK;
}

srtm_status srtm_workspace_size_tv(const srtm_shape* shape, int32_t smoother, size_t* bytes) {
  srtm_status s = check_shape(shape);
  if (s != SRTM_OK) return s;
  if (!bytes) return SRTM_E_NULL;
  if (shape->nx > srtm::TV_NX_MAX) return SRTM_E_UNSUPPORTED;
  const size_t esz = shape->dtype == SRTM_F64 ? 8 : 4;
  *bytes = srtm::make_work_layout(shape->nx, shape->ny, shape->L, shape->N, esz, smoother != 0, false, true).total;
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

srtm_status srtm_smooth_noalloc(const srtm_shape* shape, const void* F, const void* Q, const void* H,
                                const void* R, const void* m0, const void* P0, const void* y, void* ms_fast,
                                void* Ps_fast, void* ms_slow, void* Ps_slow, void* mf_fast, void* Pf_fast,
                                void* mf_slow, void* Pf_slow, int32_t* info, void* stream) {
  srtm_status s = check_shape(shape);
  if (s != SRTM_OK) return s;
  if (!F || !Q || !H || !R || !m0 || !P0 || !y) return SRTM_E_NULL;
  const size_t esz = shape->dtype == SRTM_F64 ? 8 : 4;
  if (srtm::make_work_layout(shape->nx, shape->ny, shape->L, shape->N, esz, true).total > SRTM_NOALLOC_SCRATCH_BYTES)
    return SRTM_E_SCRATCH;
  void* ws = nullptr;
  s = scratch_address(&ws);
  if (s != SRTM_OK) return s;
  const srtm::Ptrs p{F, Q, H, R, m0, P0, y, ms_fast, Ps_fast, ms_slow, Ps_slow,
                     mf_fast, Pf_fast, mf_slow, Pf_slow, ws, info};
  return run_common(shape, p, true, SRTM_NOALLOC_SCRATCH_BYTES, stream, nullptr, 0);
}

srtm_status srtm_smooth_sequential(const srtm_shape* shape, const void* F, const void* Q, const void* H,
                                   const void* R, const void* m0, const void* P0, const void* y, void* ms_fast,
                                   void* Ps_fast, void* ms_slow, void* Ps_slow, void* workspace,
                                   size_t workspace_bytes, int32_t* info, void* stream) {
  srtm_status s = check_shape(shape);
  if (s != SRTM_OK) return s;
  if (!F || !Q || !H || !R || !m0 || !P0 || !y || !workspace) return SRTM_E_NULL;
  const void* all[] = {F, Q, H, R, m0, P0, y, ms_fast, Ps_fast, ms_slow, Ps_slow};
  for (const void* q : all)
    if (!aligned(q, 16)) return SRTM_E_ALIGN;
  if (!aligned(workspace, 256) || !aligned(info, 4)) return SRTM_E_ALIGN;
  const size_t esz = shape->dtype == SRTM_F64 ? 8 : 4;
  if (workspace_bytes < srtm::make_work_layout(shape->nx, shape->ny, shape->L, shape->N, esz, true).total)
    return SRTM_E_WORKSPACE;
  const srtm::Ptrs p{F, Q, H, R, m0, P0, y, ms_fast, Ps_fast, ms_slow, Ps_slow,
                     nullptr, nullptr, nullptr, nullptr, workspace, info};
  return srtm::dispatch(*shape, p, true, static_cast<hipStream_t>(stream), nullptr, 0, srtm::REC_SEQ);
}

srtm_status srtm_smooth_lag1(const srtm_shape* shape, const void* F, const void* Q, const void* H, const void* R,
                             const void* m0, const void* P0, const void* y, void* ms_fast, void* Ps_fast,
                             void* ms_slow, void* Ps_slow, void* Cs_fast, void* workspace, size_t workspace_bytes,
                             int32_t* info, void* stream) {
  if (!Cs_fast) return SRTM_E_NULL;
  srtm::Ptrs p{F, Q, H, R, m0, P0, y, ms_fast, Ps_fast, ms_slow, Ps_slow,
               nullptr, nullptr, nullptr, nullptr, workspace, info};
  p.Cs_fast = Cs_fast;
  return run_common(shape, p, true, workspace_bytes, stream, nullptr, 0);
}

srtm_status srtm_filter_inputs(const srtm_shape* shape, const srtm_inputs* inputs, const void* F, const void* Q,
                               const void* H, const void* R, const void* m0, const void* P0, const void* y,
                               void* m_fast, void* P_fast, void* m_slow, void* P_slow, void* workspace,
                               size_t workspace_bytes, int32_t* info, void* stream) {
  srtm::Ptrs p{F, Q, H, R, m0, P0, y, nullptr, nullptr, nullptr, nullptr,
               m_fast, P_fast, m_slow, P_slow, workspace, info};
  const srtm_status s = with_inputs(inputs, p);
  if (s != SRTM_OK) return s;
  return run_common(shape, p, false, workspace_bytes, stream, nullptr, 0);
}

srtm_status srtm_smooth_inputs(const srtm_shape* shape, const srtm_inputs* inputs, const void* F, const void* Q,
                               const void* H, const void* R, const void* m0, const void* P0, const void* y,
                               void* ms_fast, void* Ps_fast, void* ms_slow, void* Ps_slow, void* mf_fast,
                               void* Pf_fast, void* mf_slow, void* Pf_slow, void* workspace,
                               size_t workspace_bytes, int32_t* info, void* stream) {
  srtm::Ptrs p{F, Q, H, R, m0, P0, y, ms_fast, Ps_fast, ms_slow, Ps_slow,
               mf_fast, Pf_fast, mf_slow, Pf_slow, workspace, info};
  const srtm_status s = with_inputs(inputs, p);
  if (s != SRTM_OK) return s;
  return run_common(shape, p, true, workspace_bytes, stream, nullptr, 0);
}

srtm_status srtm_filter_tv(const srtm_shape* shape, const void* F, const void* Q, const void* H, const void* R,
                           const void* m0, const void* P0, const void* y, void* m_fast, void* P_fast, void* m_slow,
                           void* P_slow, void* workspace, size_t workspace_bytes, int32_t* info, void* stream) {
  srtm::Ptrs p{F, Q, H, R, m0, P0, y, nullptr, nullptr, nullptr, nullptr,
               m_fast, P_fast, m_slow, P_slow, workspace, info};
  p.tv = true;
  return run_common(shape, p, false, workspace_bytes, stream, nullptr, 0);
}

srtm_status srtm_smooth_tv(const srtm_shape* shape, const void* F, const void* Q, const void* H, const void* R,
                           const void* m0, const void* P0, const void* y, void* ms_fast, void* Ps_fast,
                           void* ms_slow, void* Ps_slow, void* mf_fast, void* Pf_fast, void* mf_slow,
                           void* Pf_slow, void* workspace, size_t workspace_bytes, int32_t* info, void* stream) {
  srtm::Ptrs p{F, Q, H, R, m0, P0, y, ms_fast, Ps_fast, ms_slow, Ps_slow,
               mf_fast, Pf_fast, mf_slow, Pf_slow, workspace, info};
  p.tv = true;
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

srtm_status srtm_batch_plan(int32_t nx, int32_t ny, int32_t dtype, const srtm_seq* seqs, int32_t nseq,
                            void* table, size_t table_bytes, size_t* table_size, size_t* workspace_size,
                            int64_t* ntiles, int32_t* max_L) {
  if (!seqs || !table_size || !workspace_size || !ntiles || !max_L) return SRTM_E_NULL;
  if (nseq < 1) return SRTM_E_SHAPE;
  const size_t esz = dtype == SRTM_F64 ? 8 : 4;
  int64_t tiles = 0;
  size_t ws = 0;
  int32_t lmax = 1;
  for (int32_t s = 0; s < nseq; ++s) {
    const srtm_seq& q = seqs[s];
    const srtm_shape sh{nx, ny, q.L, (srtm_dtype)dtype, q.N};
    srtm_status st = check_shape(&sh);
    if (st != SRTM_OK) return st;
    if (q.reserved != 0) return SRTM_E_SHAPE;
    if (!q.F || !q.Q || !q.H || !q.R || !q.m0 || !q.P0 || !q.y) return SRTM_E_NULL;
    const void* all[] = {q.F, q.Q, q.H, q.R, q.m0, q.P0, q.y, q.ms_fast, q.Ps_fast, q.ms_slow, q.Ps_slow};
    for (const void* p : all)
      if (!aligned(p, 16)) return SRTM_E_ALIGN;
    tiles += (q.N + srtm::TILE - 1) / srtm::TILE;
    ws += srtm::align256(srtm::make_work_layout(nx, ny, q.L, q.N, esz, true).total);
    if (q.L > lmax) lmax = q.L;
  }
  if (tiles > INT32_MAX) return SRTM_E_UNSUPPORTED;
  const size_t map_off = srtm::batch_tile_map_offset(nseq);
  const size_t need = map_off + (size_t)tiles * sizeof(int32_t);
  *table_size = need;
  *workspace_size = ws;
  *ntiles = tiles;
  *max_L = lmax;
  if (!table || table_bytes < need) return SRTM_OK;
  srtm::SeqDesc* d = static_cast<srtm::SeqDesc*>(table);
  int32_t* map = reinterpret_cast<int32_t*>(static_cast<char*>(table) + map_off);
  int64_t t0 = 0;
  size_t off = 0;
  for (int32_t s = 0; s < nseq; ++s) {
    const srtm_seq& q = seqs[s];
    srtm::SeqDesc e{};
    e.F = q.F; e.Q = q.Q; e.H = q.H; e.R = q.R; e.m0 = q.m0; e.P0 = q.P0; e.y = q.y;
    e.ms_fast = q.ms_fast; e.Ps_fast = q.Ps_fast; e.ms_slow = q.ms_slow; e.Ps_slow = q.Ps_slow;
    e.N = q.N;
    e.tile0 = t0;
    e.ws_off = off;
    e.L = q.L;
    e.smoother = 1;
    e.nx = nx;
    e.ny = ny;
    d[s] = e;
    const int64_t nt = (q.N + srtm::TILE - 1) / srtm::TILE;
    for (int64_t t = 0; t < nt; ++t) map[t0 + t] = s;
    t0 += nt;
    off += srtm::align256(srtm::make_work_layout(nx, ny, q.L, q.N, esz, true).total);
  }
  return SRTM_OK;
}

// A batch descriptor's arrays, checked again when the table is launched (it may have been edited
// since it was planned): the model, prior and measurements present, every array 16-byte aligned.
static srtm_status check_desc_arrays(const srtm::SeqDesc& d) {
  if (!d.F || !d.Q || !d.H || !d.R || !d.m0 || !d.P0 || !d.y) return SRTM_E_NULL;
  const void* all[] = {d.F,       d.Q,       d.H,       d.R,       d.m0,      d.P0,      d.y,      d.ms_fast,
                       d.Ps_fast, d.ms_slow, d.Ps_slow, d.mf_fast, d.Pf_fast, d.mf_slow, d.Pf_slow, d.B,
                       d.u};
  for (const void* q : all)
    if (!aligned(q, 16)) return SRTM_E_ALIGN;
  return SRTM_OK;
}

static srtm_status batch_common(int32_t nx, int32_t ny, int32_t dtype, int32_t nseq, const void* table_host,
                                const void* table_dev, void* workspace, size_t workspace_bytes, int32_t* info,
                                void* stream, bool grad) {
  if (!table_host || !table_dev || !workspace) return SRTM_E_NULL;
  if (dtype != SRTM_F32 && dtype != SRTM_F64) return SRTM_E_DTYPE;
  if (nseq < 1) return SRTM_E_SHAPE;
  if (!srtm::pair_supported(nx, ny)) return SRTM_E_UNSUPPORTED;
  if (!aligned(table_dev, 16) || !aligned(workspace, 256) || !aligned(info, 4)) return SRTM_E_ALIGN;
  const size_t esz = dtype == SRTM_F64 ? 8 : 4;
  const srtm::SeqDesc* d = static_cast<const srtm::SeqDesc*>(table_host);
  int64_t tiles = 0;
  int32_t lmax = 1;
  for (int32_t s = 0; s < nseq; ++s) {
    const srtm_shape sh{nx, ny, d[s].L, (srtm_dtype)dtype, d[s].N};
    srtm_status st = check_shape(&sh);
    if (st != SRTM_OK) return st;
    if (d[s].tile0 != tiles || d[s].smoother != 1) return SRTM_E_SHAPE;
    if (d[s].B || d[s].u || d[s].nu || d[s].tv || d[s].Cs_fast)  // batches: time-invariant, no inputs
      return SRTM_E_SHAPE;
    st = check_desc_arrays(d[s]);
    if (st != SRTM_OK) return st;
    const int32_t* map = reinterpret_cast<const int32_t*>(static_cast<const char*>(table_host) +
                                                          srtm::batch_tile_map_offset(nseq));
    const int64_t nt = (d[s].N + srtm::TILE - 1) / srtm::TILE;
    for (int64_t t = 0; t < nt; ++t)
      if (map[tiles + t] != s) return SRTM_E_SHAPE;
    const size_t end = d[s].ws_off + srtm::make_work_layout(nx, ny, d[s].L, d[s].N, esz, true).total;
    if (d[s].ws_off % 256 != 0 || end > workspace_bytes) return SRTM_E_WORKSPACE;
    tiles += (d[s].N + srtm::TILE - 1) / srtm::TILE;
    if (d[s].L > lmax) lmax = d[s].L;
  }
  if (tiles > INT32_MAX) return SRTM_E_UNSUPPORTED;
  if (grad)  // the four output slots receive ll, dF, dQ, dR: all required
    for (int32_t s = 0; s < nseq; ++s)
      if (!d[s].ms_fast || !d[s].Ps_fast || !d[s].ms_slow || !d[s].Ps_slow) return SRTM_E_NULL;
  return srtm::dispatch_batch(nx, ny, dtype, table_dev, nseq, tiles, lmax, workspace, info,
                              static_cast<hipStream_t>(stream), grad);
}

srtm_status srtm_smooth_batch(int32_t nx, int32_t ny, int32_t dtype, int32_t nseq, const void* table_host,
                              const void* table_dev, void* workspace, size_t workspace_bytes, int32_t* info,
                              void* stream) {
  return batch_common(nx, ny, dtype, nseq, table_host, table_dev, workspace, workspace_bytes, info, stream, false);
}

srtm_status srtm_loglik_grad_batch(int32_t nx, int32_t ny, int32_t dtype, int32_t nseq, const void* table_host,
                                   const void* table_dev, void* workspace, size_t workspace_bytes, int32_t* info,
                                   void* stream) {
  return batch_common(nx, ny, dtype, nseq, table_host, table_dev, workspace, workspace_bytes, info, stream, true);
}

// Validates one mixed-batch sequence; its workspace block size goes to *ws.
static srtm_status check_seq_ex(int32_t dtype, const srtm_seq_ex& q, size_t* ws) {
  const srtm_shape sh{q.nx, q.ny, q.L, (srtm_dtype)dtype, q.N};
  srtm_status st = check_shape(&sh);
  if (st != SRTM_OK) return st;
  if (q.reserved != 0 || (q.per_window != 0 && q.per_window != 1)) return SRTM_E_SHAPE;
  if (!q.F || !q.Q || !q.H || !q.R || !q.m0 || !q.P0 || !q.y) return SRTM_E_NULL;
  const bool inputs = q.B || q.u || q.nu;
  if (inputs) {
    if (!q.B || !q.u) return SRTM_E_NULL;
    if (q.nu < 1 || q.nu > SRTM_MAX_NU) return SRTM_E_SHAPE;
  }
  if (q.per_window) {
    if (q.nx > srtm::TV_NX_MAX) return SRTM_E_UNSUPPORTED;
    if (inputs) return SRTM_E_SHAPE;  // per-window models take no inputs
  }
  const void* all[] = {q.F, q.Q, q.H, q.R, q.m0, q.P0, q.y, q.B, q.u, q.ms_fast, q.Ps_fast, q.ms_slow, q.Ps_slow};
  for (const void* p : all)
    if (!aligned(p, 16)) return SRTM_E_ALIGN;
  const size_t esz = dtype == SRTM_F64 ? 8 : 4;
  *ws = srtm::align256(srtm::make_work_layout(q.nx, q.ny, q.L, q.N, esz, true, inputs, q.per_window != 0).total);
  return SRTM_OK;
}

srtm_status srtm_batch_plan_ex(int32_t dtype, const srtm_seq_ex* seqs, int32_t nseq, void* table, size_t table_bytes,
                               size_t* table_size, size_t* workspace_size, int64_t* ntiles, int32_t* max_L) {
  if (!seqs || !table_size || !workspace_size || !ntiles || !max_L) return SRTM_E_NULL;
  if (dtype != SRTM_F32 && dtype != SRTM_F64) return SRTM_E_DTYPE;
  if (nseq < 1) return SRTM_E_SHAPE;
  int64_t tiles = 0;
  size_t ws = 0;
  int32_t lmax = 1;
  std::vector<size_t> block(nseq);  // each sequence's workspace block
  for (int32_t s = 0; s < nseq; ++s) {
    const srtm_status st = check_seq_ex(dtype, seqs[s], &block[s]);
    if (st != SRTM_OK) return st;
    tiles += (seqs[s].N + srtm::TILE - 1) / srtm::TILE;
    ws += block[s];
    if (seqs[s].L > lmax) lmax = seqs[s].L;
  }
  if (tiles > INT32_MAX) return SRTM_E_UNSUPPORTED;
  const size_t map_off = srtm::batch_tile_map_offset(nseq);
  const size_t need = map_off + (size_t)tiles * sizeof(int32_t);
  *table_size = need;
  *workspace_size = ws;
  *ntiles = tiles;
  *max_L = lmax;
  if (!table || table_bytes < need) return SRTM_OK;
  srtm::SeqDesc* d = static_cast<srtm::SeqDesc*>(table);
  int32_t* map = reinterpret_cast<int32_t*>(static_cast<char*>(table) + map_off);
  int64_t t0 = 0;
  size_t off = 0;
  for (int32_t s = 0; s < nseq; ++s) {
    const srtm_seq_ex& q = seqs[s];
    srtm::SeqDesc e{};
    e.F = q.F; e.Q = q.Q; e.H = q.H; e.R = q.R; e.m0 = q.m0; e.P0 = q.P0; e.y = q.y;
    e.ms_fast = q.ms_fast; e.Ps_fast = q.Ps_fast; e.ms_slow = q.ms_slow; e.Ps_slow = q.Ps_slow;
    e.N = q.N;
    e.tile0 = t0;
    e.ws_off = off;
    e.L = q.L;
    e.smoother = 1;
    e.B = q.B;
    e.u = q.u;
    e.nu = q.B ? q.nu : 0;
    e.tv = q.per_window;
    e.nx = q.nx;
    e.ny = q.ny;
    d[s] = e;
    const int64_t nt = (q.N + srtm::TILE - 1) / srtm::TILE;
    for (int64_t t = 0; t < nt; ++t) map[t0 + t] = s;
    t0 += nt;
    off += block[s];
  }
  return SRTM_OK;
}

srtm_status srtm_smooth_batch_ex(int32_t dtype, int32_t nseq, const void* table_host, const void* table_dev,
                                 void* workspace, size_t workspace_bytes, int32_t* info, void* stream) {
  if (!table_host || !table_dev || !workspace) return SRTM_E_NULL;
  if (dtype != SRTM_F32 && dtype != SRTM_F64) return SRTM_E_DTYPE;
  if (nseq < 1) return SRTM_E_SHAPE;
  if (!aligned(table_dev, 16) || !aligned(workspace, 256) || !aligned(info, 4)) return SRTM_E_ALIGN;
  const size_t esz = dtype == SRTM_F64 ? 8 : 4;
  const srtm::SeqDesc* d = static_cast<const srtm::SeqDesc*>(table_host);
  const int32_t* map =
      reinterpret_cast<const int32_t*>(static_cast<const char*>(table_host) + srtm::batch_tile_map_offset(nseq));
  int64_t tiles = 0;
  int32_t lmax = 1;
  for (int32_t s = 0; s < nseq; ++s) {
    const srtm_shape sh{d[s].nx, d[s].ny, d[s].L, (srtm_dtype)dtype, d[s].N};
    srtm_status st = check_shape(&sh);
    if (st != SRTM_OK) return st;
    if (d[s].tile0 != tiles || d[s].smoother != 1 || d[s].Cs_fast) return SRTM_E_SHAPE;
    const bool inputs = d[s].B != nullptr;
    if (inputs != (d[s].u != nullptr) || (inputs ? (d[s].nu < 1 || d[s].nu > SRTM_MAX_NU) : d[s].nu != 0))
      return SRTM_E_SHAPE;
    if (d[s].tv != 0 && (d[s].tv != 1 || inputs || d[s].nx > srtm::TV_NX_MAX)) return SRTM_E_SHAPE;
    st = check_desc_arrays(d[s]);
    if (st != SRTM_OK) return st;
    const int64_t nt = (d[s].N + srtm::TILE - 1) / srtm::TILE;
    for (int64_t t = 0; t < nt; ++t)
      if (map[tiles + t] != s) return SRTM_E_SHAPE;
    const size_t end =
        d[s].ws_off + srtm::make_work_layout(d[s].nx, d[s].ny, d[s].L, d[s].N, esz, true, inputs, d[s].tv != 0).total;
    if (d[s].ws_off % 256 != 0 || end > workspace_bytes) return SRTM_E_WORKSPACE;
    tiles += nt;
    if (d[s].L > lmax) lmax = d[s].L;
  }
  if (tiles > INT32_MAX) return SRTM_E_UNSUPPORTED;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  return dtype == SRTM_F64 ? srtm::run_mixed_double(d, table_dev, nseq, tiles, lmax, workspace, info, st)
                           : srtm::run_mixed_float(d, table_dev, nseq, tiles, lmax, workspace, info, st);
}

srtm_status srtm_graph_begin(void* stream) {
  if (!stream) return SRTM_E_NULL;
  return hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeRelaxed) == hipSuccess
             ? SRTM_OK
             : SRTM_E_HIP;
}

srtm_status srtm_graph_end(void* stream, void** exec) {
  if (!stream || !exec) return SRTM_E_NULL;
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(static_cast<hipStream_t>(stream), &g) != hipSuccess || !g) return SRTM_E_HIP;
  hipGraphExec_t e = nullptr;
  const hipError_t r = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (r != hipSuccess || !e) return SRTM_E_HIP;
  *exec = e;
  return SRTM_OK;
}

srtm_status srtm_graph_launch(void* exec, void* stream) {
  if (!exec) return SRTM_E_NULL;
  return hipGraphLaunch(static_cast<hipGraphExec_t>(exec), static_cast<hipStream_t>(stream)) == hipSuccess
             ? SRTM_OK
             : SRTM_E_HIP;
}

srtm_status srtm_graph_destroy(void* exec) {
  if (!exec) return SRTM_E_NULL;
  return hipGraphExecDestroy(static_cast<hipGraphExec_t>(exec)) == hipSuccess ? SRTM_OK : SRTM_E_HIP;
}

static srtm_status lik_common(const srtm_shape* shape, const void* F, const void* Q, const void* H, const void* R,
                              const void* m0, const void* P0, const void* y, void* ll, void* dF, void* dQ, void* dR,
                              void* workspace, size_t workspace_bytes, int32_t* info, void* stream, bool grad,
                              const srtm_inputs* inputs = nullptr) {
  srtm_status s = check_shape(shape);
  if (s != SRTM_OK) return s;
  if (!F || !Q || !H || !R || !m0 || !P0 || !y || !ll || !workspace) return SRTM_E_NULL;
  if (grad && (!dF || !dQ || !dR)) return SRTM_E_NULL;
  const void* all[] = {F, Q, H, R, m0, P0, y, ll, dF, dQ, dR};
  for (const void* q : all)
    if (!aligned(q, 16)) return SRTM_E_ALIGN;
  if (!aligned(workspace, 256) || !aligned(info, 4)) return SRTM_E_ALIGN;
  const size_t esz = shape->dtype == SRTM_F64 ? 8 : 4;
  if (workspace_bytes <
      srtm::make_work_layout(shape->nx, shape->ny, shape->L, shape->N, esz, grad, inputs != nullptr).total)
    return SRTM_E_WORKSPACE;
  srtm::Ptrs p{F, Q, H, R, m0, P0, y, nullptr, nullptr, nullptr, nullptr,
               nullptr, nullptr, nullptr, nullptr, workspace, info};
  if (inputs) {
    const srtm_status si = with_inputs(inputs, p);
    if (si != SRTM_OK) return si;
  }
  return srtm::dispatch(*shape, p, grad, static_cast<hipStream_t>(stream), nullptr, 0,
                        grad ? srtm::REC_GRAD : srtm::REC_LL, ll, dF, dQ, dR);
}

srtm_status srtm_loglik(const srtm_shape* shape, const void* F, const void* Q, const void* H, const void* R,
                        const void* m0, const void* P0, const void* y, void* ll, void* workspace,
                        size_t workspace_bytes, int32_t* info, void* stream) {
  return lik_common(shape, F, Q, H, R, m0, P0, y, ll, nullptr, nullptr, nullptr, workspace, workspace_bytes, info,
                    stream, false);
}

srtm_status srtm_loglik_inputs(const srtm_shape* shape, const srtm_inputs* inputs, const void* F, const void* Q,
                               const void* H, const void* R, const void* m0, const void* P0, const void* y,
                               void* ll, void* workspace, size_t workspace_bytes, int32_t* info, void* stream) {
  if (!inputs) return SRTM_E_NULL;
  return lik_common(shape, F, Q, H, R, m0, P0, y, ll, nullptr, nullptr, nullptr, workspace, workspace_bytes, info,
                    stream, false, inputs);
}

srtm_status srtm_loglik_grad(const srtm_shape* shape, const void* F, const void* Q, const void* H, const void* R,
                             const void* m0, const void* P0, const void* y, void* ll, void* dF, void* dQ, void* dR,
                             void* workspace, size_t workspace_bytes, int32_t* info, void* stream) {
  return lik_common(shape, F, Q, H, R, m0, P0, y, ll, dF, dQ, dR, workspace, workspace_bytes, info, stream, true);
}

srtm_status srtm_loglik_grad_inputs(const srtm_shape* shape, const srtm_inputs* inputs, const void* F, const void* Q,
                                    const void* H, const void* R, const void* m0, const void* P0, const void* y,
                                    void* ll, void* dF, void* dQ, void* dR, void* workspace, size_t workspace_bytes,
                                    int32_t* info, void* stream) {
  if (!inputs) return SRTM_E_NULL;
  return lik_common(shape, F, Q, H, R, m0, P0, y, ll, dF, dQ, dR, workspace, workspace_bytes, info, stream, true,
                    inputs);
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
    case SRTM_E_SCRATCH: return "srtm_smooth_noalloc: workspace larger than SRTM_NOALLOC_SCRATCH_BYTES";
    default: return "unknown status";
  }
}

int32_t srtm_version(void) { return 100; }

}  // extern "C"
