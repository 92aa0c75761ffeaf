// Layout of the per-call constants block and of the workspace (host and device).
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace srtm {

constexpr int TILE = 256;       // windows per workgroup in the per-tile kernels
constexpr int LOG_TILE = 8;
constexpr int KS = 256;         // threads of the Kogge-Stone tile-level scans
constexpr int LOG_KS = 8;

inline __host__ __device__ int ceil_log2(int64_t x) {
  int l = 0;
  while ((int64_t(1) << l) < x) ++l;
  return l;
}

// Tile-level forward scan plan: each of the KS threads folds `chunk` (a power of two)
// tiles, `active` threads take part in ceil_log2(active) Kogge-Stone steps, and the
// constants kernel provides scan levels 0 .. nlev-1 (segments of 2^p windows): the in-tile
// levels below LOG_TILE, the chunk level LOG_TILE + lchunk that the prior is folded with, and
// one level per step above it (levels LOG_TILE + lchunk .. + steps - 1).
struct ScanPlan {
  int64_t nt;
  int lchunk, active, steps, nlev;
};

inline __host__ __device__ ScanPlan make_scan_plan(int64_t N) {
  ScanPlan s;
  s.nt = (N + TILE - 1) / TILE;
  s.lchunk = ceil_log2((s.nt + KS - 1) / KS);
  s.active = (int)((s.nt + (int64_t(1) << s.lchunk) - 1) >> s.lchunk);
  s.steps = ceil_log2(s.active);
  const int need = LOG_TILE + s.lchunk + (s.steps > 0 ? s.steps : 1);
  s.nlev = need > LOG_TILE + 1 ? need : LOG_TILE + 1;
  return s;
}

// Offsets (in scalars) into the constants block written by the constants kernel.
struct ConstLayout {
  int nx, ny, L;
  int A, Q, Cbar, Rx, K, Heta;   // model and slow-rate constants
  int per_i, per_i_stride;       // per fast step i = 1..L: A^i, Q_ii, Q_iL, c_i
  int o_Ai, o_Qii, o_QiL, o_ci;
  int lev, lev_stride;           // per level p: F, D, J of 2^p merged windows and
  int o_F, o_D, o_J, o_G1, o_G2, o_G3, o_G4;  // the vector-combine coefficients
  int total;
};

inline __host__ __device__ ConstLayout make_const_layout(int nx, int ny, int L, int nlev = 0) {
  ConstLayout c;
  const int nn = nx * nx, nxy = nx * ny;
  c.nx = nx; c.ny = ny; c.L = L;
  int o = 0;
  c.A = o; o += nn;
  c.Q = o; o += nn;
  c.Cbar = o; o += nxy;
  c.Rx = o; o += ny * ny;
  c.K = o; o += nxy;
  c.Heta = o; o += nxy;
  o = (o + 7) & ~7;
  c.o_Ai = 0; c.o_Qii = nn; c.o_QiL = 2 * nn; c.o_ci = 3 * nn;
  c.per_i_stride = (3 * nn + nxy + 7) & ~7;
  c.per_i = o; o += L * c.per_i_stride;
  c.o_F = 0; c.o_D = nn; c.o_J = 2 * nn;
  c.o_G1 = 3 * nn; c.o_G2 = 4 * nn; c.o_G3 = 5 * nn; c.o_G4 = 6 * nn;
  c.lev_stride = (7 * nn + 7) & ~7;
  c.lev = o; o += nlev * c.lev_stride;
  c.total = o;
  return c;
}

// Dynamic LDS of the constants kernel (float64 per-step tables and level-chain scratch).
inline __host__ __device__ size_t constants_lds_bytes(int nx, int ny, int L) {
  const int nn = nx * nx, nxy = nx * ny;
  const int w2s = nn > 2 * nxy ? nn : 2 * nxy;
  return sizeof(double) * (size_t)(2 * nn + nxy + ny * ny + (L + 1) * (3 * nn + w2s + nxy) + 19 * nn);
}

// Workspace regions, byte offsets (256-byte aligned).
struct WorkLayout {
  size_t consts, consts64, chain, ftile_agg, ftile_state, utree, carry, btile_agg, btile_state, sfx, stats, inp, tvblk, tvel,
      total;
};

// Time-varying (per-window) models: offsets (in scalars) into one window's constants block.
// Window-level: C_bar, R_x, K, Heta = C_bar^T R_x^{-1}, A^l and c_l. Then the backward factors of
// the fast steps, A^s and C Sig_s with s = l - i and Sig_s = sum_{u<=s} A^u (Q_il = Q_ii (A^s)^T,
// c_i = (1/l) [a_i + Q_ii (C Sig_s)^T] run backwards in i), for even s only: slot q = 0 ..
// ceil(l/2)-1 holds A^{2q} and C Sig_{2q}; the odd s = 2q+1 follows as A A^{2q} and
// C Sig_{2q} + C A^{2q+1}. The recovery forms A^i, Q_ii and a_i by forward recursions from the
// window's own A, Q and C.
struct TvLayout {
  int Cbar, Rx, K, Heta, AL, cL;
  int slot, slot_stride, o_As, o_CS;
  int total;
};

inline __host__ __device__ TvLayout make_tv_layout(int nx, int ny, int L) {
  TvLayout t;
  const int nn = nx * nx, nxy = nx * ny;
  int o = 0;
  t.Cbar = o; o += nxy;
  t.Rx = o; o += ny * ny;
  t.K = o; o += nxy;
  t.Heta = o; o += nxy;
  t.AL = o; o += nn;
  t.cL = o; o += nxy;
  t.o_As = 0; t.o_CS = nn;
  t.slot_stride = nn + nxy;
  t.slot = o; o += ((L + 1) / 2) * t.slot_stride;
  t.total = o;
  return t;
}

// Scalars of one window's constants block and of its element record (F, D, J).
inline __host__ __device__ int tv_block_size(int nx, int ny, int L) { return make_tv_layout(nx, ny, L).total; }
inline __host__ __device__ constexpr int tv_elem_size(int nx) { return 3 * nx * nx; }

// Scalars (float64) of one tile's log-likelihood / gradient record.
inline __host__ __device__ constexpr int stat_size(int nx, int ny) { return 1 + 2 * nx * nx + ny * ny; }

// Per-window smoother-correction record: Et (nx^2), gt (nx), St (upper triangle).
inline __host__ __device__ constexpr int sfx_stride(int nx) { return nx * nx + nx + nx * (nx + 1) / 2; }

inline __host__ __device__ size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// `utree` (time-invariant models): the tile reductions' up-sweep trees, per tile 2 nx rows of TILE
// scalars, which the per-tile forward pass reloads instead of repeating the up-sweep.
// `inputs`: the call has known inputs, whose per-window record (y_k - mu_k, z_{k,l}) [N][ny + nx]
// the tile reductions write for the later kernels. `tv`: the model is given per window; the
// per-window constants blocks [N][tv_block_size] and element records [N][tv_elem_size] follow,
// and the tile aggregates of the forward scan are whole elements.
inline __host__ __device__ WorkLayout make_work_layout(int nx, int ny, int L, int64_t N, size_t esz, bool smoother,
                                                       bool inputs = false, bool tv = false) {
  WorkLayout w;
  const ConstLayout c = make_const_layout(nx, ny, L, make_scan_plan(N).nlev);
  const int64_t nt = (N + TILE - 1) / TILE;
  const size_t nn = (size_t)nx * nx;
  const size_t fagg = tv ? (size_t)(3 * nn + 2 * nx) : (size_t)(2 * nx);  // scalars per tile aggregate
  size_t o = 0;
  w.consts = o; o = align256(o + (size_t)c.total * esz);
  w.consts64 = o; o = align256(o + (size_t)c.lev * sizeof(double));  // float64 copy of the model part
  w.chain = o; o = align256(o + 3 * nn * sizeof(double));  // float64 F, D, J handed between launches
  w.ftile_agg = o; o = align256(o + (size_t)nt * fagg * esz);
  w.ftile_state = o; o = align256(o + (size_t)nt * (nx + nn) * esz);
  if (!tv) {
    w.utree = o; o = align256(o + (size_t)nt * TILE * 2 * nx * esz);
  } else {
    w.utree = 0;
  }
  w.carry = o; o = align256(o + (size_t)N * (nx + nn) * esz);
  if (smoother) {
    w.btile_agg = o; o = align256(o + (size_t)nt * (2 * nn + nx) * esz);
    w.btile_state = o; o = align256(o + (size_t)nt * (nx + nn) * esz);
    w.sfx = o; o = align256(o + (size_t)N * sfx_stride(nx) * esz);
  } else {
    w.btile_agg = w.btile_state = w.sfx = 0;
  }
  w.stats = o; o = align256(o + (size_t)nt * stat_size(nx, ny) * sizeof(double));
  if (inputs) {
    w.inp = o; o = align256(o + (size_t)N * (nx + ny) * esz);
  } else {
    w.inp = 0;
  }
  if (tv) {  // stored tile by tile (whole tiles)
    w.tvblk = o; o = align256(o + (size_t)nt * TILE * tv_block_size(nx, ny, L) * esz);
    w.tvel = o; o = align256(o + (size_t)nt * TILE * tv_elem_size(nx) * esz);
  } else {
    w.tvblk = w.tvel = 0;
  }
  w.total = o;
  return w;
}

// One sequence of a call: device pointers of its model, data and outputs (typed by the call's
// dtype; outputs nullable), its place in the call's tile numbering and its workspace block.
struct SeqDesc {
  const void *F, *Q, *H, *R, *m0, *P0, *y;
  void *ms_fast, *Ps_fast, *ms_slow, *Ps_slow, *mf_fast, *Pf_fast, *mf_slow, *Pf_slow;
  int64_t N;
  int64_t tile0;     // first tile of the sequence among the call's tiles
  uint64_t ws_off;   // byte offset of the sequence's workspace block (256-byte aligned)
  int32_t L;
  int32_t smoother;  // the block holds the smoother regions
  const void *B, *u;  // known inputs (null without)
  int32_t nu;
  int32_t tv;  // F, Q, H, R are given per window ([N][...])
  void* Cs_fast;  // lag-one smoothed cross-covariances [N][L][nx][nx] (single calls only; null otherwise)
  int32_t nx, ny;  // the sequence's sizes (the mixed-pair kernels dispatch on them)
};

// What every kernel receives: either one sequence (`table` null) or a device table of
// sequences with the sequence index of every tile.
struct Batch {
  const SeqDesc* table;
  const int32_t* tile_seq;
  char* ws;
  int32_t* info;  // one status word per sequence, nullable
  SeqDesc one;
};

// Byte offset of the tile-to-sequence map behind nseq descriptors in a batch table.
inline __host__ __device__ size_t batch_tile_map_offset(int nseq) {
  return (((size_t)nseq * sizeof(SeqDesc)) + 15) & ~size_t(15);
}

}  // namespace srtm
