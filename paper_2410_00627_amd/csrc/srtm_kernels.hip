// HIP kernels for parallel-in-time SRTM filtering and smoothing on gfx950.
//
// Method: Yaghoobi & Sarkka, arXiv 2410.00627, Sec. IV. The forward pass is the
// parallel IMKF: an inclusive scan of the filter elements (eq. a-k-f) under the
// operator of eq. op-filter, which yields the slow-rate carry (m^f_{k,l}, P^f_{k,l}).
// The reverse pass is the parallel IMS: a suffix scan of the smoother elements
// (eq. parallel-ak-smoothing) under eq. op-smoother, which yields (m^s_{k,1}, P^s_{k,1}),
// followed by the per-window fast-rate recovery of eq. seq-smoothing-all
// (Remarks fast-par-filter and parallel-fast-smoothing).
//
// Design points specific to this implementation (the paper's equations are unchanged):
//  * The model is time invariant, so every filter element with k > 1 shares its matrix
//    part (F, D, J); a run of 2^p consecutive elements therefore has matrices that depend
//    on p only. The constants kernel computes them once per call (repeated squaring under
//    eq. op-filter), and the per-tile up-sweeps combine only the vector parts (d, eta)
//    with per-level coefficient matrices shared by every lane.
//  * The first element is written as a prior state (0, m0, P0, 0, 0) combined with the
//    generic element of window 1; this equals the paper's a_1 = (0, m^f_{1,l}, P^f_{1,l}).
//  * A prefix that contains the prior has F = 0, so every exclusive prefix is a "state"
//    (m, P) and the down-sweeps combine states with aligned segments.
//  * The suffix scan is a Kogge-Stone scan towards lower window indices inside a tile and,
//    at tile level, a Kogge-Stone scan over the tiles counted from the end; a suffix that
//    reaches the last window has E = 0 and is the smoothed state itself.
//  * Within a window only the blocks the outputs need are formed (Remark
//    cross-covariances): P^f_{k,i,i}, P^f_{k,i,l} and means, from per-step constants
//    A^i, Q_ii, Q_il, c_i, instead of the dense (l nx)^2 window covariance.
//  * Models given per window (time varying) share nothing between elements: their kernels
//    (k_tv_*) build each window's constants and element in one lane and scan whole elements.

#include <hip/hip_ext.h>

#include <type_traits>

#include "srtm_device.h"
#include "srtm_entry.h"
#include "srtm_layout.h"

namespace srtm {

// Every array of a call is device (global) memory. Pointers read from a descriptor are
// generic; passing them through the global address space lets the compiler emit global
// instead of flat loads and stores.
template <typename T>
SRTM_DEV T* as_global(T* p) {
  using G = __attribute__((address_space(1))) T*;
  return (T*)((G)p);
}
template <typename T>
SRTM_DEV T* as_global(const void* p) {
  return as_global(static_cast<T*>(const_cast<void*>(p)));
}

// Store of one scalar to device memory through a global pointer.
template <typename T>
SRTM_DEV void put_global(T* p, T v) {
  *(__attribute__((address_space(1))) T*)p = v;
}

// Staged copy of n scalars with the nthr threads of a workgroup: value q = ld(q) is handed to
// st(q, value). Each thread issues up to B loads before its first store.
template <int B, typename T, class LD, class ST>
SRTM_DEV void staged_copy(int n, int tid, int nthr, LD ld, ST st) {
#pragma unroll 1
  for (int base = 0; base < n; base += B * nthr) {
    T v[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int q = base + i * nthr + tid;
      v[i] = (q < n) ? ld(q) : T(0);
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int q = base + i * nthr + tid;
      if (q < n) st(q, v[i]);
    }
  }
}

// ============================================================================ constants
// Cofactor (r, c) of the NX x NX row-major matrix M: (-1)^{r+c} times the determinant of M
// without row r and column c.
template <int NX>
SRTM_DEV double cofactor(const double* M, int r, int c) {
  constexpr int K = NX - 1;
  if constexpr (K == 0) {
    return 1.0;
  } else {
    double a[K][K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      const int ri = i < r ? i : i + 1;
#pragma unroll
      for (int j = 0; j < K; ++j) a[i][j] = M[ri * NX + (j < c ? j : j + 1)];
    }
    double d;
    if constexpr (K == 1) {
      d = a[0][0];
    } else if constexpr (K == 2) {
      d = a[0][0] * a[1][1] - a[0][1] * a[1][0];
    } else {
      d = a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0]) +
          a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]);
    }
    return ((r + c) & 1) ? -d : d;
  }
}

// Level chain over levels p0 .. p1-1, run by wave 0 of a workgroup (one lane per matrix entry).
// `chain` is 19 nx^2 doubles of LDS whose first 3 nx^2 hold F, D, J of Theta(2^p0). Writes the
// level records p0 .. p1-1 and, when p1 < nlev, F, D, J of Theta(2^p1) in float64 to `hand`
// (3 nx^2 doubles), where a continuation of the chain in a later launch picks them up.
//   Theta(2^{p+1}) = Theta(2^p) (x) Theta(2^p) under eq. op-filter, W = (I + D J)^{-1}, and the
// coefficients that combine the vector parts of two runs of 2^p elements:
//   d_ij = G1 d_i + G2 eta_j + d_j,   eta_ij = G3 eta_j - G4 d_i + eta_i,
//   G1 = F W, G2 = F W D, G3 = (W F)^T, G4 = (W F)^T J.
// W is the adjugate of I + D J over its determinant, with one cofactor per lane (nx <= 4).
template <typename T, int NX>
SRTM_DEV int level_chain(double* chain, T* __restrict__ cst, const ConstLayout& lay, int p0, int p1, int nlev,
                         double* __restrict__ hand) {
  constexpr int NN = NX * NX;
  double* rec = chain;
  double* nrec = chain + 7 * NN;
  double* sM = chain + 14 * NN;
  double* sCof = sM + NN;
  double* sW = sCof + NN;
  double* sWF = sW + NN;
  double* sXD = sWF + NN;
  int lflag = 0;
  const int e = threadIdx.x;
  for (int p = p0; p < p1; ++p) {
    const double* F = rec;
    const double* D = rec + NN;
    const double* J = rec + 2 * NN;
    for (int o = e; o < NN; o += 64) {  // M = I + D J
      const int er = o / NX, ec = o % NX;
      double acc = (er == ec) ? 1.0 : 0.0;
      for (int k = 0; k < NX; ++k) acc += D[er * NX + k] * J[k * NX + ec];
      sM[o] = acc;
    }
    wave_sync();
    if constexpr (NX <= 4) {
      if (e < NN) sCof[e] = cofactor<NX>(sM, e / NX, e % NX);
      wave_sync();
      if (e < NN) {  // W = adj(M) / det(M), adj(M)[r][c] = C[c][r]
        double det = 0.0;
        for (int c = 0; c < NX; ++c) det += sM[c] * sCof[c];
        const double id = rcp_nr(det);
        if (e == 0 && !(det != 0.0 && isfinite(id))) lflag |= SRTM_INFO_COMBINE_SINGULAR;
        sW[e] = sCof[(e % NX) * NX + e / NX] * id;
      }
    } else {  // larger states: one lane, Gaussian elimination with partial pivoting
      if (e == 0) {
        double Mr[NX][NX], Wr[NX][NX];
        for (int r = 0; r < NX; ++r)
          for (int c = 0; c < NX; ++c) Mr[r][c] = sM[r * NX + c];
        if (!inv_small(Mr, Wr)) lflag |= SRTM_INFO_COMBINE_SINGULAR;
        for (int r = 0; r < NX; ++r)
          for (int c = 0; c < NX; ++c) sW[r * NX + c] = Wr[r][c];
      }
    }
    wave_sync();
    // The three products of each phase are formed by three groups of lanes with the same
    // instructions (operands chosen by pointer and stride, no divergent branches):
    //   WF = W F, G1 = F W, XD = sym(W D);
    for (int q = e; q < 3 * NN; q += 64) {
      const int part = q / NN, o = q % NN, er = o / NX, ec = o % NX;
      const double* X = part == 1 ? F : sW;
      const double* Y = part == 0 ? F : (part == 1 ? sW : D);
      double t1 = 0.0, t2 = 0.0;
      for (int k = 0; k < NX; ++k) {
        t1 += X[er * NX + k] * Y[k * NX + ec];
        t2 += X[ec * NX + k] * Y[k * NX + er];
      }
      double* dst = part == 0 ? sWF + o : (part == 1 ? rec + 3 * NN + o : sXD + o);
      *dst = part == 2 ? 0.5 * (t1 + t2) : t1;
    }
    wave_sync();
    //   G2 = F XD, G4 = (WF)^T J, next F = F WF; and G3 = (WF)^T;
    for (int q = e; q < 3 * NN; q += 64) {
      const int part = q / NN, o = q % NN, er = o / NX, ec = o % NX;
      const double* X = part == 1 ? sWF : F;
      const int xr = part == 1 ? 1 : NX, xk = part == 1 ? NX : 1;
      const double* Y = part == 0 ? sXD : (part == 1 ? J : sWF);
      double acc = 0.0;
      for (int k = 0; k < NX; ++k) acc += X[er * xr + k * xk] * Y[k * NX + ec];
      double* dst = part == 0 ? rec + 4 * NN + o : (part == 1 ? rec + 6 * NN + o : nrec + o);
      *dst = acc;
      if (part == 0) rec[5 * NN + ec * NX + er] = sWF[o];
    }
    wave_sync();
    //   next D = sym(G2 F^T) + D, next J = sym(G4 F) + J.
    for (int q = e; q < 2 * NN; q += 64) {
      const int part = q / NN, o = q % NN, er = o / NX, ec = o % NX;
      const double* X = rec + (part == 0 ? 4 : 6) * NN;
      const int yk = part == 0 ? 1 : NX, yc = part == 0 ? NX : 1;
      double t1 = 0.0, t2 = 0.0;
      for (int k = 0; k < NX; ++k) {
        t1 += X[er * NX + k] * F[k * yk + ec * yc];
        t2 += X[ec * NX + k] * F[k * yk + er * yc];
      }
      nrec[(1 + part) * NN + o] = 0.5 * (t1 + t2) + rec[(1 + part) * NN + o];
    }
    T* dst = cst + lay.lev + p * lay.lev_stride;  // the level record, as laid out in LDS
    for (int q = e; q < 7 * NN; q += 64) dst[q] = (T)rec[q];
    wave_sync();
    double* t = rec;
    rec = nrec;
    nrec = t;
  }
  if (p1 < nlev) {
    for (int q = threadIdx.x; q < 3 * NN; q += 64) put_global(hand + q, rec[q]);
  }
  return lflag;
}

// Levels 0 .. CHAIN_SPLIT-1 come from the constants kernel (the in-tile scans need the levels
// below LOG_TILE); the rest, which only the tile-level scan uses, from one workgroup of the
// tile-reduction launch, so that they are computed while the tiles are reduced (for 2^17 windows
// nine levels, about 12 us in float64, beside reductions of about 10 us; a level costs about 0.9 us
// more in the constants kernel, so a higher split does not pay).
constexpr int CHAIN_SPLIT = LOG_TILE;
static_assert(CHAIN_SPLIT >= LOG_TILE, "the tile reductions read levels below LOG_TILE");

// Dynamic LDS of the tile-reduction launch: the larger of a tile reduction's slots and level
// coefficients and a level chain's float64 scratch.
template <typename T, int NX>
constexpr size_t fwd_reduce_lds_bytes() {
  constexpr size_t red = sizeof(T) * (size_t)(2 * NX * TILE + LOG_TILE * 4 * NX * NX);
  constexpr size_t chn = sizeof(double) * (size_t)(19 * NX * NX);
  return red > chn ? red : chn;
}

// The rest of the level chain (levels CHAIN_SPLIT .. nlev-1), continued from the handed-over
// Theta(2^CHAIN_SPLIT). The wave runs at raised priority: it shares its SIMD with reductions.
template <typename T, int NX, int NY>
SRTM_DEV void chain_tail_body(T* __restrict__ cst, const double* __restrict__ hand, int L, int nlev,
                              int32_t* info) {
  constexpr int NN = NX * NX;
  extern __shared__ char smraw[];
  double* chain = reinterpret_cast<double*>(smraw);  // 19 nx^2 (fwd_reduce_lds_bytes)
  const int tid = threadIdx.x;
  if (tid >= 64 || nlev <= CHAIN_SPLIT) return;
  __builtin_amdgcn_s_setprio(3);
  for (int q = tid; q < 3 * NN; q += 64) chain[q] = gld(hand + q);
  wave_sync();
  const ConstLayout lay = make_const_layout(NX, NY, L, nlev);
  const int f = level_chain<T, NX>(chain, cst, lay, CHAIN_SPLIT, nlev, nlev, nullptr);
  if (f && info) atomicOr(info, f);
}

// One workgroup, float64 throughout. Per-step tables are built in LDS by parallel
// loops; the slow-rate constants and the level tables by the lanes of wave 0.
//
// With Q_ij = Cov(x_{k,i}, x_{k,j} | x_{k-1,l}) = sum_{t=1..min(i,j)} A^{i-t} Q A^{(j-t)T}:
//   Q_ii = sum_{t=0}^{i-1} A^t Q A^{tT},   Q_il = Q_ii (A^{l-i})^T,
//   c_i  = (1/l) sum_j Q_ij C^T = Cov(x_{k,i}, y_k | x_{k-1,l})  (noise part),
//   C_bar = (C/l) sum_{i=1..l} A^i,  R_x = (1/l) sum_i C c_i + R,  G_bar Q~ M_bar^T = c_l,
//   Q_bar = Q_ll, A_bar = A^l   (eq. h-k-l-2, eq. y-k-l-2 and eq. a-k-f).
template <typename T, int NX, int NY>
SRTM_DEV void constants_body(const T* __restrict__ Fm, const T* __restrict__ Qm, const T* __restrict__ Hm,
                             const T* __restrict__ Rm, int L, int nlev, T* __restrict__ cst,
                             double* __restrict__ cst64, double* __restrict__ hand, int32_t* info) {
  constexpr int NN = NX * NX, NXY = NX * NY;
  constexpr int W2S = (NN > 2 * NXY ? NN : 2 * NXY);
  extern __shared__ double sm[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const ConstLayout lay = make_const_layout(NX, NY, L, nlev);
  double* sA = sm;
  double* sQ = sA + NN;
  double* sC = sQ + NN;
  double* sR = sC + NXY;
  double* Apow = sR + NY * NY;          // (L+1) NN, Apow[i] = A^i
  double* Qii = Apow + (L + 1) * NN;    // (L+1) NN, Qii[i] = Q_ii (Qii[0] = 0)
  double* W1 = Qii + (L + 1) * NN;      // (L+1) NN scratch
  double* W2 = W1 + (L + 1) * NN;       // (L+1) W2S scratch
  double* ci = W2 + (L + 1) * W2S;      // (L+1) NXY, ci[i] = c_i
  double* chain = ci + (L + 1) * NXY;   // 19 NN: level-chain records and scratch

  for (int e = tid; e < NN; e += nthr) {
    sA[e] = (double)Fm[e];
    sQ[e] = (double)Qm[e];
    Apow[e] = (e / NX == e % NX) ? 1.0 : 0.0;
    Apow[NN + e] = (double)Fm[e];
  }
  for (int e = tid; e < NXY; e += nthr) sC[e] = (double)Hm[e];
  for (int e = tid; e < NY * NY; e += nthr) sR[e] = (double)Rm[e];
  __syncthreads();

  // A^i by doubling: A^i = A^s A^{i-s} for i in (s, 2s].
  for (int s = 1; s < L; s *= 2) {
    const int hi = (2 * s < L) ? 2 * s : L;
    for (int e = tid; e < (hi - s) * NN; e += nthr) {
      const int i = s + 1 + e / NN, rc = e % NN, r = rc / NX, c = rc % NX;
      double acc = 0.0;
      for (int k = 0; k < NX; ++k) acc += Apow[s * NN + r * NX + k] * Apow[(i - s) * NN + k * NX + c];
      Apow[i * NN + rc] = acc;
    }
    __syncthreads();
  }
  // W2[t] = A^t Q A^tT, t = 0..L-1: one entry of the upper triangle per item, mirrored, so that
  // every sum of these blocks is exactly symmetric.
  for (int e = tid; e < L * NN; e += nthr) {
    const int t = e / NN, rc = e % NN, r = rc / NX, c = rc % NX;
    if (c < r) continue;
    const double* At = Apow + t * NN;
    double acc = 0.0;
    for (int k = 0; k < NX; ++k) {
      double aq = 0.0;
      for (int j = 0; j < NX; ++j) aq += At[r * NX + j] * sQ[j * NX + k];
      acc += aq * At[c * NX + k];
    }
    W2[t * NN + r * NX + c] = acc;
    W2[t * NN + c * NX + r] = acc;
  }
  __syncthreads();
  // Q_ii = sum_{t<i} W2[t] (Qii[0] = 0) and W1[s] = Sig_s = sum_{u=0}^{s} A^u. Item (i, rc) forms
  // entry rc of Q_{i+1,i+1} (i < l) and of Sig_i, each as four independent partial sums (a
  // running sum would chain one LDS round trip per term).
  auto sum_blocks = [&](const double* src, int n, int rc) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int t = 0;
    for (; t + 4 <= n; t += 4) {
      a0 += src[t * NN + rc];
      a1 += src[(t + 1) * NN + rc];
      a2 += src[(t + 2) * NN + rc];
      a3 += src[(t + 3) * NN + rc];
    }
    for (; t < n; ++t) a0 += src[t * NN + rc];
    return (a0 + a1) + (a2 + a3);
  };
  for (int e = tid; e < (L + 1) * NN; e += nthr) {
    const int i = e / NN, rc = e % NN;
    if (i < L) Qii[(i + 1) * NN + rc] = sum_blocks(W2, i + 1, rc);
    if (i == 0) Qii[rc] = 0.0;
    W1[i * NN + rc] = sum_blocks(Apow, i + 1, rc);
  }
  __syncthreads();
  // CS[s] = C Sig_s (NY x NX) in W2[0 ..], QC[j] = Q_jj C^T (NX x NY) in W2[(L+1) NXY ..]; beside
  // them the per-step tables go to the constants block: A^i, Q_ii, Q_il = Q_ii (A^{l-i})^T, and
  // A, Q. Every entry of the model part (below the level tables) also goes, unrounded, to the
  // float64 copy.
  double* CS = W2;
  double* QC = W2 + (L + 1) * NXY;
  auto put = [&](int off, double v) {
    cst[off] = (T)v;
    cst64[off] = v;
  };
  for (int e = tid; e < (L + 1) * NXY + (L + 1) * NN; e += nthr) {
    if (e < (L + 1) * NXY) {
      const int s = e / NXY, rc = e % NXY;
      {
        const int r = rc / NX, c = rc % NX;  // CS: NY x NX
        double acc = 0.0;
        for (int k = 0; k < NX; ++k) acc += sC[r * NX + k] * W1[s * NN + k * NX + c];
        CS[s * NXY + rc] = acc;
      }
      {
        const int r = rc / NY, c = rc % NY;  // QC: NX x NY
        double acc = 0.0;
        for (int k = 0; k < NX; ++k) acc += Qii[s * NN + r * NX + k] * sC[c * NX + k];
        QC[s * NXY + rc] = acc;
      }
    } else if (e < (L + 1) * NXY + L * NN) {
      const int e2 = e - (L + 1) * NXY;
      const int i = 1 + e2 / NN, rc = e2 % NN, r = rc / NX, c = rc % NX;
      const int base = lay.per_i + (i - 1) * lay.per_i_stride;
      put(base + lay.o_Ai + rc, Apow[i * NN + rc]);
      put(base + lay.o_Qii + rc, Qii[i * NN + rc]);
      double acc = 0.0;
      for (int k = 0; k < NX; ++k) acc += Qii[i * NN + r * NX + k] * Apow[(L - i) * NN + c * NX + k];
      put(base + lay.o_QiL + rc, acc);
    } else {
      const int q = e - (L + 1) * NXY - L * NN;
      put(lay.A + q, sA[q]);
      put(lay.Q + q, sQ[q]);
    }
  }
  __syncthreads();
  // c_i = (1/l) [ sum_{j<i} A^{i-j} Q_jj C^T + Q_ii (C Sig_{l-i})^T ], the sum over j as four
  // independent partial sums.
  for (int e = tid; e < L * NXY; e += nthr) {
    const int i = 1 + e / NXY, rc = e % NXY, r = rc / NY, c = rc % NY;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int k = 0; k < NX; ++k) a0 += Qii[i * NN + r * NX + k] * CS[(L - i) * NXY + c * NX + k];
    int j = 1;
    for (; j + 4 <= i; j += 4)
      for (int k = 0; k < NX; ++k) {
        a0 += Apow[(i - j) * NN + r * NX + k] * QC[j * NXY + k * NY + c];
        a1 += Apow[(i - j - 1) * NN + r * NX + k] * QC[(j + 1) * NXY + k * NY + c];
        a2 += Apow[(i - j - 2) * NN + r * NX + k] * QC[(j + 2) * NXY + k * NY + c];
        a3 += Apow[(i - j - 3) * NN + r * NX + k] * QC[(j + 3) * NXY + k * NY + c];
      }
    for (; j < i; ++j)
      for (int k = 0; k < NX; ++k) a0 += Apow[(i - j) * NN + r * NX + k] * QC[j * NXY + k * NY + c];
    ci[i * NXY + rc] = ((a0 + a1) + (a2 + a3)) / (double)L;
  }
  __syncthreads();

  // c_i to the constants block; C_bar = (C/l)(Sig_l - I) and R_x = (1/l) sum_i C c_i + R into LDS
  // (W2 is free again).
  double* sCbar = W2;
  double* sRx = W2 + NXY;
  for (int e = tid; e < L * NXY + NXY + NY * NY; e += nthr) {
    if (e < L * NXY) {
      const int i = 1 + e / NXY, rc = e % NXY;
      put(lay.per_i + (i - 1) * lay.per_i_stride + lay.o_ci + rc, ci[i * NXY + rc]);
    } else if (e < L * NXY + NXY) {
      const int q = e - L * NXY, r = q / NX, c = q % NX;
      double acc = 0.0;
      for (int k = 0; k < NX; ++k) acc += sC[r * NX + k] * (W1[L * NN + k * NX + c] - (k == c ? 1.0 : 0.0));
      sCbar[q] = acc / (double)L;
    } else {
      const int q = e - L * NXY - NXY, r = q / NY, c = q % NY;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int i = 1;
      for (; i + 4 <= L + 1; i += 4)
        for (int k = 0; k < NX; ++k) {
          a0 += sC[r * NX + k] * ci[i * NXY + k * NY + c];
          a1 += sC[r * NX + k] * ci[(i + 1) * NXY + k * NY + c];
          a2 += sC[r * NX + k] * ci[(i + 2) * NXY + k * NY + c];
          a3 += sC[r * NX + k] * ci[(i + 3) * NXY + k * NY + c];
        }
      for (; i <= L; ++i)
        for (int k = 0; k < NX; ++k) a0 += sC[r * NX + k] * ci[i * NXY + k * NY + c];
      sRx[q] = ((a0 + a1) + (a2 + a3)) / (double)L + sR[r * NY + c];
    }
  }
  __syncthreads();
  if (tid >= 64) return;  // the rest is done by wave 0
  int lflag = 0;
  double* rec = chain;  // the chain's F, D, J of Theta(1): the generic element
  {
    // ------------------------------------------------------------ generic element (wave 0)
    // Every lane inverts R_x itself; lane e < nx^2 forms entry e of F, D and J (D and J from
    // both halves, symmetrised), and the first lanes write C_bar, R_x, K and H_eta.
    //   K = S_xy R_x^{-1},  H_eta = C_bar^T R_x^{-1},  F = A^l - K C_bar,
    //   D = Q_ll - K S_xy^T,  J = H_eta C_bar,  with S_xy = c_l.
    double Rx[NY][NY], Rxi[NY][NY];
    for (int r = 0; r < NY; ++r)
      for (int c = 0; c < NY; ++c) Rx[r][c] = sRx[r * NY + c];
    symmetrize(Rx);
    if (!spd_inv(Rx, Rxi) && tid == 0) lflag |= SRTM_INFO_INNOVATION_NOT_PD;
    const double* Sxy = ci + L * NXY;  // NX x NY
    auto krow = [&](int r, double (&o)[NY]) {  // row r of K
#pragma unroll
      for (int k = 0; k < NY; ++k) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NY; ++j) s += Sxy[r * NY + j] * Rxi[j][k];
        o[k] = s;
      }
    };
    auto hrow = [&](int r, double (&o)[NY]) {  // row r of H_eta
#pragma unroll
      for (int k = 0; k < NY; ++k) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NY; ++j) s += sCbar[j * NX + r] * Rxi[j][k];
        o[k] = s;
      }
    };
    if (tid < NN) {
      const int r = tid / NX, c = tid % NX;
      double Kr[NY], Kc[NY], Hr[NY], Hc[NY];
      krow(r, Kr);
      krow(c, Kc);
      hrow(r, Hr);
      hrow(c, Hc);
      double f = Apow[L * NN + tid], drc = Qii[L * NN + r * NX + c], dcr = Qii[L * NN + c * NX + r];
      double jrc = 0.0, jcr = 0.0;
#pragma unroll
      for (int k = 0; k < NY; ++k) {
        f -= Kr[k] * sCbar[k * NX + c];
        drc -= Kr[k] * Sxy[c * NY + k];
        dcr -= Kc[k] * Sxy[r * NY + k];
        jrc += Hr[k] * sCbar[k * NX + c];
        jcr += Hc[k] * sCbar[k * NX + r];
      }
      rec[tid] = f;
      rec[NN + tid] = (r == c) ? drc : 0.5 * (drc + dcr);
      rec[2 * NN + tid] = (r == c) ? jrc : 0.5 * (jrc + jcr);
    }
    if (tid < NX) {
      double Kr[NY], Hr[NY];
      krow(tid, Kr);
      hrow(tid, Hr);
#pragma unroll
      for (int k = 0; k < NY; ++k) {
        put(lay.K + tid * NY + k, Kr[k]);
        put(lay.Heta + tid * NY + k, Hr[k]);
      }
    }
    for (int q = tid; q < NXY; q += 64) put(lay.Cbar + q, sCbar[q]);
    for (int q = tid; q < NY * NY; q += 64) {
      const int r = q / NY, c = q % NY;
      put(lay.Rx + q, (r == c) ? sRx[q] : 0.5 * (sRx[r * NY + c] + sRx[c * NY + r]));
    }
  }
  wave_sync();
  // Levels below CHAIN_SPLIT; the others continue in the tile-reduction launch.
  const int p1 = nlev < CHAIN_SPLIT ? nlev : CHAIN_SPLIT;
  lflag |= level_chain<T, NX>(chain, cst, lay, 0, p1, nlev, hand);
  if (lflag && info) atomicOr(info, lflag);
}

// ============================================================================ helpers
// Known inputs of a call (all null and nu = 0 without inputs).
template <typename T>
struct InputView {
  const T* B;  // [nx][nu]
  const T* u;  // [N][l][nu], u[k-1][i-1] drives x_{k,i}
  const T* H;  // [ny][nx], the measurement matrix C
  T* rec;      // workspace [N][ny + nx]: y_k - mu_k and z_{k,l}, written by the tile reductions
  int nu;
};

// A call's constants block (time-invariant model).
template <typename T, int NX, int NY>
struct Model {
  const T* __restrict__ cst;
  ConstLayout lay;
  InputView<T> in{};
  SRTM_DEV const T* per_i(int i) const { return cst + lay.per_i + (i - 1) * lay.per_i_stride; }
  SRTM_DEV int per_i_off(int i) const { return lay.per_i + (i - 1) * lay.per_i_stride; }
  SRTM_DEV const T* level(int p) const { return cst + lay.lev + p * lay.lev_stride; }
  SRTM_DEV int AL_off(int L) const { return per_i_off(L) + lay.o_Ai; }  // A^l
  SRTM_DEV int cL_off(int L) const { return per_i_off(L) + lay.o_ci; }  // c_l
  template <int R, int C>
  SRTM_DEV void get(T (&a)[R][C], int off) const { load(a, cst + off); }
  SRTM_DEV T at(int off) const { return cst[off]; }
};

// Per-window blocks and element records are stored tile by tile, window-minor within a tile:
// scalar j of window k at base[(k / TILE) * width * TILE + j * TILE + k % TILE] for records of
// `width` scalars, so that the lanes of a wave read and write consecutive addresses and one
// tile's records stay within width * TILE scalars. Returns window k's column (stride TILE).
template <typename T>
SRTM_DEV T* tv_column(T* base, int64_t k, int width) {
  return base + (k / TILE) * (int64_t)width * TILE + (k % TILE);
}
// The block of columns of window k's tile (tv_column minus the column).
template <typename T>
SRTM_DEV T* tv_tile_base(T* base, int64_t k, int width) {
  return base + (k / TILE) * (int64_t)width * TILE;
}

// One window of a per-window model: its constants block (TvLayout, one column of its tile's
// block of columns at `blk`: the row base blk + off * TILE is the same for every lane of a
// workgroup and each lane adds its column) and its own A, Q and C, entry j at A[j * ms]: the
// caller's row-major arrays (LDSM false, ms = 1) or a window-minor copy in LDS (LDSM, ms the
// copy's column count).
template <typename T, int NX, int NY, bool LDSM = false>
struct TvModel {
  const T* __restrict__ blk;
  TvLayout lay;
  int lane;
  const T* __restrict__ A;
  const T* __restrict__ Q;
  const T* __restrict__ C;
  int ms = 1;
  SRTM_DEV T mdl(const T* p, int j) const { return LDSM ? sld(p + j * ms) : gld(p + j * ms); }
  SRTM_DEV int AL_off(int) const { return lay.AL; }
  SRTM_DEV int cL_off(int) const { return lay.cL; }
  SRTM_DEV int slot_off(int q) const { return lay.slot + q * lay.slot_stride; }
  template <int R, int CC>
  SRTM_DEV void get(T (&a)[R][CC], int off) const {
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < CC; ++c) a[r][c] = at(off + r * CC + c);
  }
  SRTM_DEV T at(int off) const { return gld(blk + (int64_t)off * TILE + lane); }
};

template <typename T, int N>
SRTM_DEV T symget(const T (&P)[N][N], int r, int c) { return r <= c ? P[r][c] : P[c][r]; }

// state (m, P) (x) segment (F, d, D, eta, J): the eq. op-filter combination whose left
// operand holds the prior (F = 0):  W = (I + P J)^{-1},
//   m' = F W (m + P eta) + d,   P' = F W P F^T + D   (W P is symmetric; its upper triangle is used).
template <typename T, int NX>
SRTM_DEV bool state_combine(T (&m)[NX], T (&P)[NX][NX], const T (&F)[NX][NX], const T (&d)[NX],
                            const T (&D)[NX][NX], const T (&eta)[NX], const T (&J)[NX][NX]) {
  T M[NX][NX], W[NX][NX];
  mm(P, J, M);
#pragma unroll
  for (int r = 0; r < NX; ++r) M[r][r] += T(1);
  const bool ok = inv_small(M, W);
  T u[NX], Wu[NX], WP[NX][NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T t = m[r];
#pragma unroll
    for (int k = 0; k < NX; ++k) t = my_fma(P[r][k], eta[k], t);
    u[r] = t;
  }
  mv(W, u, Wu);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = r; c < NX; ++c) {
      T t = T(0);
#pragma unroll
      for (int k = 0; k < NX; ++k) t = my_fma(W[r][k], P[k][c], t);
      WP[r][c] = t;
      WP[c][r] = t;
    }
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T t = d[r];
#pragma unroll
    for (int k = 0; k < NX; ++k) t = my_fma(F[r][k], Wu[k], t);
    m[r] = t;
  }
  sandwich(F, WP, D, P);
  return ok;
}

// Full filter element and a_i (x) a_j of eq. op-filter, with W = (I + D_i J_j)^{-1} and
// (I + J_j D_i)^{-1} = W^T (D, J symmetric):
//   F = F_j W F_i, d = F_j W (d_i + D_i eta_j) + d_j, D = F_j W D_i F_j^T + D_j,
//   eta = (W F_i)^T (eta_j - J_j d_i) + eta_i,  J = (W F_i)^T J_j F_i + J_i.
template <typename T, int NX>
struct FElem {
  T F[NX][NX], d[NX], D[NX][NX], e[NX], J[NX][NX];
};

template <typename T, int NX>
SRTM_DEV bool elem_combine(const FElem<T, NX>& a, const FElem<T, NX>& b, FElem<T, NX>& o) {
  T M[NX][NX], W[NX][NX];
  mm(a.D, b.J, M);
#pragma unroll
  for (int r = 0; r < NX; ++r) M[r][r] += T(1);
  const bool ok = inv_small(M, W);
  T XF[NX][NX], u[NX], Xu[NX], XD[NX][NX];
  mm(W, a.F, XF);
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T t = a.d[r];
#pragma unroll
    for (int k = 0; k < NX; ++k) t = my_fma(a.D[r][k], b.e[k], t);
    u[r] = t;
  }
  mv(W, u, Xu);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = r; c < NX; ++c) {
      T t = T(0);
#pragma unroll
      for (int k = 0; k < NX; ++k) t = my_fma(W[r][k], a.D[k][c], t);
      XD[r][c] = t;
      XD[c][r] = t;
    }
  FElem<T, NX> t;
  mm(b.F, XF, t.F);
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T q = b.d[r];
#pragma unroll
    for (int k = 0; k < NX; ++k) q = my_fma(b.F[r][k], Xu[k], q);
    t.d[r] = q;
  }
  sandwich(b.F, XD, b.D, t.D);
  T vv[NX], JF[NX][NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T q = b.e[r];
#pragma unroll
    for (int k = 0; k < NX; ++k) q = my_fma(-b.J[r][k], a.d[k], q);
    vv[r] = q;
  }
  mm(b.J, a.F, JF);
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T q = a.e[r];
#pragma unroll
    for (int k = 0; k < NX; ++k) q = my_fma(XF[k][r], vv[k], q);
    t.e[r] = q;
#pragma unroll
    for (int c = r; c < NX; ++c) {
      T sj = a.J[r][c];
#pragma unroll
      for (int k = 0; k < NX; ++k) sj = my_fma(XF[k][r], JF[k][c], sj);
      t.J[r][c] = sj;
      t.J[c][r] = sj;
    }
  }
  o = t;
  return ok;
}

template <typename T, int NX>
SRTM_DEV void elem_identity(FElem<T, NX>& a) {
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    a.d[r] = T(0);
    a.e[r] = T(0);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      a.F[r][c] = (r == c) ? T(1) : T(0);
      a.D[r][c] = T(0);
      a.J[r][c] = T(0);
    }
  }
}

// Smoother element (E, g, S) and eq. op-smoother: for a (earlier) and b (later),
//   E = E_a E_b, g = E_a g_b + g_a, S = E_a S_b E_a^T + S_a.
template <typename T, int NX>
struct SElem {
  T E[NX][NX], g[NX], S[NX][NX];
};

template <typename T, int NX>
SRTM_DEV void selem_combine(const SElem<T, NX>& a, const SElem<T, NX>& b, SElem<T, NX>& o) {
  SElem<T, NX> t;
  mm(a.E, b.E, t.E);
  T ES[NX][NX];
  mm(a.E, b.S, ES);
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T s = a.g[r];
#pragma unroll
    for (int k = 0; k < NX; ++k) s = my_fma(a.E[r][k], b.g[k], s);
    t.g[r] = s;
#pragma unroll
    for (int c = r; c < NX; ++c) {
      T q = a.S[r][c];
#pragma unroll
      for (int k = 0; k < NX; ++k) q = my_fma(ES[r][k], a.E[c][k], q);
      t.S[r][c] = q;
      t.S[c][r] = q;
    }
  }
  o = t;
}

// segment (E, g, S) applied to the smoothed state after it: m' = E m + g, P' = E P E^T + S.
template <typename T, int NX>
SRTM_DEV void sstate_combine(const SElem<T, NX>& a, T (&m)[NX], T (&P)[NX][NX]) {
  T EP[NX][NX], mn[NX];
  mm(a.E, P, EP);
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T s = a.g[r];
#pragma unroll
    for (int k = 0; k < NX; ++k) s = my_fma(a.E[r][k], m[k], s);
    mn[r] = s;
  }
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    m[r] = mn[r];
#pragma unroll
    for (int c = r; c < NX; ++c) {
      T q = a.S[r][c];
#pragma unroll
      for (int k = 0; k < NX; ++k) q = my_fma(EP[r][k], a.E[c][k], q);
      P[r][c] = q;
      P[c][r] = q;
    }
  }
}

// ---------------------------------------------------------------- LDS slot storage (SoA)
template <typename T>
struct Slots {
  T* base;
  int n;  // slots per field row
  SRTM_DEV T& at(int f, int s) const { return base[f * n + s]; }
};

template <typename T, int NX>
SRTM_DEV void st_state(const Slots<T>& S, int s, const T (&m)[NX], const T (&P)[NX][NX]) {
#pragma unroll
  for (int r = 0; r < NX; ++r) S.at(r, s) = m[r];
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = r; c < NX; ++c) S.at(NX + r * NX + c, s) = P[r][c];
}
template <typename T, int NX>
SRTM_DEV void ld_state(const Slots<T>& S, int s, T (&m)[NX], T (&P)[NX][NX]) {
#pragma unroll
  for (int r = 0; r < NX; ++r) m[r] = S.at(r, s);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = r; c < NX; ++c) {
      P[r][c] = S.at(NX + r * NX + c, s);
      P[c][r] = P[r][c];
    }
}
template <typename T, int NX>
SRTM_DEV void st_felem(const Slots<T>& S, int s, const FElem<T, NX>& a) {
  constexpr int NN = NX * NX;
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    S.at(NN + r, s) = a.d[r];
    S.at(2 * NN + NX + r, s) = a.e[r];
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      S.at(r * NX + c, s) = a.F[r][c];
      S.at(NN + NX + r * NX + c, s) = a.D[r][c];
      S.at(2 * NN + 2 * NX + r * NX + c, s) = a.J[r][c];
    }
  }
}
template <typename T, int NX>
SRTM_DEV void ld_felem(const Slots<T>& S, int s, FElem<T, NX>& a) {
  constexpr int NN = NX * NX;
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    a.d[r] = S.at(NN + r, s);
    a.e[r] = S.at(2 * NN + NX + r, s);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      a.F[r][c] = S.at(r * NX + c, s);
      a.D[r][c] = S.at(NN + NX + r * NX + c, s);
      a.J[r][c] = S.at(2 * NN + 2 * NX + r * NX + c, s);
    }
  }
}
template <typename T, int NX>
SRTM_DEV void st_selem(const Slots<T>& S, int s, const SElem<T, NX>& a) {
  constexpr int NN = NX * NX;
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    S.at(NN + r, s) = a.g[r];
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      S.at(r * NX + c, s) = a.E[r][c];
      S.at(NN + NX + r * NX + c, s) = a.S[r][c];
    }
  }
}
template <typename T, int NX>
SRTM_DEV void ld_selem(const Slots<T>& S, int s, SElem<T, NX>& a) {
  constexpr int NN = NX * NX;
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    a.g[r] = S.at(NN + r, s);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      a.E[r][c] = S.at(r * NX + c, s);
      a.S[r][c] = S.at(NN + NX + r * NX + c, s);
    }
  }
}

// x <- x (x) b under eq. op-smoother, where b is the element of lane l + d (DOWN) or l - d of the
// same wave, when `take`; otherwise x is left as it is. Every lane takes part in the exchange.
// The partner's E and S arrive column by column and are consumed at once, so that only a few
// exchanged values are live (the products are those of selem_combine, in its order).
template <bool DOWN, typename T, int NX>
SRTM_DEV void selem_merge_lane(SElem<T, NX>& x, int d, bool take) {
  auto mv = [&](T v) { return DOWN ? __shfl_down(v, (unsigned)d, 64) : __shfl_up(v, (unsigned)d, 64); };
  T tE[NX][NX], ES[NX][NX], tg[NX];
#pragma unroll
  for (int c = 0; c < NX; ++c) {
    T be[NX], bs[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      be[k] = mv(x.E[k][c]);
      bs[k] = mv(x.S[k][c]);
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      T e = x.E[r][0] * be[0], q = x.E[r][0] * bs[0];
#pragma unroll
      for (int k = 1; k < NX; ++k) {
        e = my_fma(x.E[r][k], be[k], e);
        q = my_fma(x.E[r][k], bs[k], q);
      }
      tE[r][c] = e;
      ES[r][c] = q;
    }
  }
  {
    T bg[NX];
#pragma unroll
    for (int k = 0; k < NX; ++k) bg[k] = mv(x.g[k]);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      T t = x.g[r];
#pragma unroll
      for (int k = 0; k < NX; ++k) t = my_fma(x.E[r][k], bg[k], t);
      tg[r] = t;
    }
  }
  if (take) {
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = r; c < NX; ++c) {
        T q = x.S[r][c];
#pragma unroll
        for (int k = 0; k < NX; ++k) q = my_fma(ES[r][k], x.E[c][k], q);
        x.S[r][c] = q;
        x.S[c][r] = q;
      }
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      x.g[r] = tg[r];
#pragma unroll
      for (int c = 0; c < NX; ++c) x.E[r][c] = tE[r][c];
    }
  }
}

// ---------------------------------------------------------------- per-window quantities
// Window k with prior (m, P) = (m^f_{k-1,l}, P^f_{k-1,l}) and measurement y_k. With
// V = P C_bar^T, S = C_bar V + R_x, U_i = A^i V + c_i = Cov(x_{k,i}, y_k | y_{1:k-1}):
//   m^f_{k,i} = A^i m + U_i S^{-1} e,   e = y_k - C_bar m,
//   P^f_{k,i,i} = A^i P A^{iT} + Q_ii - U_i S^{-1} U_i^T,
//   P^f_{k,i,l} = A^i P A^{lT} + Q_il - U_i S^{-1} U_l^T          (eq. update-fast, blockwise).
template <typename T, int NX, int NY>
struct Window {
  T m[NX];         // prior mean (of x_{k,0})
  T mp[NX];        // m' = m + V S^{-1} e      ->  m^f_i = A^i m' + c_i Se
  T Se[NY];        // S^{-1} e
  T P[NX][NX];     // prior covariance (symmetric)
  T V[NX][NY];     // P C_bar^T
  T Si[NY][NY];    // S^{-1} (symmetric)
  T Y1[NX][NX];    // P A^{lT} - V Y2      ->  P^f_{i,l} = A^i Y1 + Q_il - c_i Y2
  T Y2[NY][NX];    // S^{-1} U_l^T
};

// MV: Model (one constants block) or TvModel (the window's own block).
template <typename T, int NX, int NY, class MV>
SRTM_DEV bool window_setup(const MV& M, int L, const T (&m)[NX], const T (&P)[NX][NX],
                           const T (&yk)[NY], Window<T, NX, NY>& w) {
  T Cb[NY][NX], Rx[NY][NY];
  M.get(Cb, M.lay.Cbar);
  M.get(Rx, M.lay.Rx);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) w.P[r][c] = P[r][c];
  mm_nt(P, Cb, w.V);
  T S[NY][NY];
  mm(Cb, w.V, S);
#pragma unroll
  for (int r = 0; r < NY; ++r)
#pragma unroll
    for (int c = 0; c < NY; ++c) S[r][c] += Rx[r][c];
  symmetrize(S);
  const bool ok = spd_inv(S, w.Si);
  T e[NY];
#pragma unroll
  for (int r = 0; r < NY; ++r) {
    T s = yk[r];
#pragma unroll
    for (int k = 0; k < NX; ++k) s = my_fma(-Cb[r][k], m[k], s);
    e[r] = s;
  }
  mv(w.Si, e, w.Se);
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    w.m[r] = m[r];
    T s = m[r];
#pragma unroll
    for (int k = 0; k < NY; ++k) s = my_fma(w.V[r][k], w.Se[k], s);
    w.mp[r] = s;
  }
  // U_l = A^l V + c_l, Y2 = S^{-1} U_l^T, Y1 = P A^{lT} - V Y2
  T AL[NX][NX], cL[NX][NY];
  M.get(AL, M.AL_off(L));
  M.get(cL, M.cL_off(L));
  T UL[NX][NY];
  mm(AL, w.V, UL);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NY; ++c) UL[r][c] += cL[r][c];
  mm_nt(w.Si, UL, w.Y2);
  T PAL[NX][NX];
  mm_nt(P, AL, PAL);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      T s = PAL[r][c];
#pragma unroll
      for (int k = 0; k < NY; ++k) s = my_fma(-w.V[r][k], w.Y2[k][c], s);
      w.Y1[r][c] = s;
    }
  return ok;
}

// Filter blocks of fast step i: mean, P^f_{i,i} and (optionally) P^f_{i,l}, from the step's
// A^i and c_i and entries (r, c) of Q_ii and Q_il given by qii(r, c) and qil(r, c).
template <bool CROSS, typename T, int NX, int NY, class QII, class QIL>
SRTM_DEV void step_blocks(const Window<T, NX, NY>& w, const T (&Ai)[NX][NX], const T (&ci)[NX][NY], QII qii,
                          QIL qil, T (&mf)[NX], T (&Pii)[NX][NX], T (&PiL)[NX][NX]) {
  // mean
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T s = T(0);
#pragma unroll
    for (int k = 0; k < NX; ++k) s = my_fma(Ai[r][k], w.mp[k], s);
#pragma unroll
    for (int k = 0; k < NY; ++k) s = my_fma(ci[r][k], w.Se[k], s);
    mf[r] = s;
  }
  // U_i = A^i V + c_i ; US = U_i S^{-1}
  T U[NX][NY], US[NX][NY];
  mm(Ai, w.V, U);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NY; ++c) U[r][c] += ci[r][c];
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NY; ++c) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < NY; ++k) s = my_fma(U[r][k], symget(w.Si, k, c), s);
      US[r][c] = s;
    }
  // P^f_{i,i} = (A^i P) A^{iT} + Q_ii - US U^T  (upper triangle, mirrored)
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T AP[NX];
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      T s = T(0);
#pragma unroll
      for (int k = 0; k < NX; ++k) s = my_fma(Ai[r][k], symget(w.P, k, c), s);
      AP[c] = s;
    }
#pragma unroll
    for (int c = r; c < NX; ++c) {
      T s = qii(r, c);
#pragma unroll
      for (int k = 0; k < NX; ++k) s = my_fma(AP[k], Ai[c][k], s);
#pragma unroll
      for (int k = 0; k < NY; ++k) s = my_fma(-US[r][k], U[c][k], s);
      Pii[r][c] = s;
      Pii[c][r] = s;
    }
  }
  if (CROSS) {
    // P^f_{i,l} = A^i Y1 + Q_il - c_i Y2
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        T s = qil(r, c);
#pragma unroll
        for (int k = 0; k < NX; ++k) s = my_fma(Ai[r][k], w.Y1[k][c], s);
#pragma unroll
        for (int k = 0; k < NY; ++k) s = my_fma(-ci[r][k], w.Y2[k][c], s);
        PiL[r][c] = s;
      }
  }
}

// Time-invariant model: the step's tables from the constants block (wave-uniform loads).
template <typename T, int NX, int NY, bool CROSS>
SRTM_DEV void window_step(const Model<T, NX, NY>& M, const Window<T, NX, NY>& w, int i, T (&mf)[NX],
                          T (&Pii)[NX][NX], T (&PiL)[NX][NX]) {
  const int po = M.per_i_off(i);
  T Ai[NX][NX], ci[NX][NY];
  M.get(Ai, po + M.lay.o_Ai);
  M.get(ci, po + M.lay.o_ci);
  step_blocks<CROSS>(
      w, Ai, ci, [&](int r, int c) { return M.at(po + M.lay.o_Qii + r * NX + c); },
      [&](int r, int c) { return M.at(po + M.lay.o_QiL + r * NX + c); }, mf, Pii, PiL);
}

// Per-window model: the fast steps of window k in order, in the prior-inclusive form. With the
// window's prior (m, P) of x_{k,0} and Sig_i = Cov(x_{k,i} | y_{1:k-1}) = A^i P A^{iT} + Q_ii,
//   Sig_i = A Sig_{i-1} A^T + Q (Sig_0 = P),  mu_i = A mu_{i-1} (mu_0 = m),
//   al_i = A (al_{i-1} + Sig_{i-1} C^T) (al_1 = 0),
//   U_i = Cov(x_{k,i}, y_k | y_{1:k-1}) = (1/l) [al_i + Sig_i (C Sig_{l-i})^T],
//   m^f_{k,i} = mu_i + U_i S^{-1} e,  P^f_{k,i,i} = Sig_i - U_i S^{-1} U_i^T,
//   P^f_{k,i,l} = Sig_i (A^{l-i})^T - U_i S^{-1} U_l^T
// (the same blocks as step_blocks: A^i P A^{lT} + Q_il = Sig_i (A^{l-i})^T), from the window's own
// A, Q and C and the backward factors A^s and C Sig_s (s = l - i) of its block, stored for even s
// (TvLayout): a step with odd s forms them from the slot it shares with step i + 1.
template <typename T, int NX, int NY>
struct TvSteps {
  T Sg[NX][NX], al[NX][NY], mu[NX];  // Sg: upper triangle only
  T fCS[NY][NX], fAs[NX][NX];        // the factors of the slot in use: C Sig_{2q}, A^{2q}
  int i = 0;  // the last step formed
  template <bool CROSS, bool LDSM>
  SRTM_DEV void next(const TvModel<T, NX, NY, LDSM>& M, int L, const Window<T, NX, NY>& w, T (&mf)[NX],
                     T (&Pii)[NX][NX], T (&PiL)[NX][NX]) {
    const int s = L - (i + 1);
    if (i == 0 || (s & 1)) {  // the first step, or the first of the two steps of slot s / 2
      const int so = M.slot_off(s >> 1);
      M.get(fCS, so + M.lay.o_CS);
      M.get(fAs, so + M.lay.o_As);
    }
    T CS[NY][NX], As[NX][NX], A[NX][NX], C[NY][NX];
#pragma unroll
    for (int r = 0; r < NX; ++r) {
#pragma unroll
      for (int c = 0; c < NX; ++c) A[r][c] = M.mdl(M.A, r * NX + c);
    }
#pragma unroll
    for (int r = 0; r < NY; ++r) {
#pragma unroll
      for (int c = 0; c < NX; ++c) C[r][c] = M.mdl(M.C, r * NX + c);
    }
    if (s & 1) {  // A^s = A A^{s-1},  C Sig_s = C Sig_{s-1} + C A^s
      mm(A, fAs, As);
#pragma unroll
      for (int r = 0; r < NY; ++r)
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          T v = fCS[r][c];
#pragma unroll
          for (int q = 0; q < NX; ++q) v = my_fma(C[r][q], As[q][c], v);
          CS[r][c] = v;
        }
    } else {
#pragma unroll
      for (int r = 0; r < NX; ++r) {
#pragma unroll
        for (int c = 0; c < NX; ++c) As[r][c] = fAs[r][c];
#pragma unroll
        for (int c = 0; c < NY; ++c) CS[c][r] = fCS[c][r];
      }
    }
    if (i == 0) {
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        mu[r] = w.m[r];
#pragma unroll
        for (int c = r; c < NX; ++c) Sg[r][c] = w.P[r][c];
#pragma unroll
        for (int c = 0; c < NY; ++c) al[r][c] = T(0);
      }
    } else {
      T b[NX][NY];
#pragma unroll
      for (int r = 0; r < NX; ++r)
#pragma unroll
        for (int c = 0; c < NY; ++c) {
          T v = al[r][c];
#pragma unroll
          for (int q = 0; q < NX; ++q) v = my_fma(symget(Sg, r, q), C[c][q], v);
          b[r][c] = v;
        }
      mm(A, b, al);
    }
    {  // Sig_i = A Sig_{i-1} A^T + Q, mu_i = A mu_{i-1}
      T AS[NX][NX], nm[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        T t = T(0);
#pragma unroll
        for (int q = 0; q < NX; ++q) t = my_fma(A[r][q], mu[q], t);
        nm[r] = t;
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          T v = T(0);
#pragma unroll
          for (int q = 0; q < NX; ++q) v = my_fma(A[r][q], symget(Sg, q, c), v);
          AS[r][c] = v;
        }
      }
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        mu[r] = nm[r];
#pragma unroll
        for (int c = r; c < NX; ++c) {
          T v = M.mdl(M.Q, r * NX + c);
#pragma unroll
          for (int q = 0; q < NX; ++q) v = my_fma(AS[r][q], A[c][q], v);
          Sg[r][c] = v;
        }
      }
    }
    ++i;
    // U = (1/l) (al + Sig C Sig_{l-i}^T),  US = U S^{-1}
    const T il = T(1) / T(L);
    T U[NX][NY], US[NX][NY];
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NY; ++c) {
        T v = al[r][c];
#pragma unroll
        for (int q = 0; q < NX; ++q) v = my_fma(symget(Sg, r, q), CS[c][q], v);
        U[r][c] = v * il;
      }
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NY; ++c) {
        T v = T(0);
#pragma unroll
        for (int q = 0; q < NY; ++q) v = my_fma(U[r][q], symget(w.Si, q, c), v);
        US[r][c] = v;
      }
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      T v = mu[r];
#pragma unroll
      for (int q = 0; q < NY; ++q) v = my_fma(U[r][q], w.Se[q], v);
      mf[r] = v;
#pragma unroll
      for (int c = r; c < NX; ++c) {
        T t = Sg[r][c];
#pragma unroll
        for (int q = 0; q < NY; ++q) t = my_fma(-US[r][q], U[c][q], t);
        Pii[r][c] = t;
        Pii[c][r] = t;
      }
    }
    if (CROSS) {
#pragma unroll
      for (int r = 0; r < NX; ++r)
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          T v = T(0);
#pragma unroll
          for (int q = 0; q < NX; ++q) v = my_fma(symget(Sg, r, q), As[c][q], v);
#pragma unroll
          for (int q = 0; q < NY; ++q) v = my_fma(-U[r][q], w.Y2[q][c], v);
          PiL[r][c] = v;
        }
    }
  }
};

// Blocks of fast step 1 (the smoother element's): from the constants block, or from the
// window's own model.
template <typename T, int NX, int NY>
SRTM_DEV void first_step(const Model<T, NX, NY>& M, int, const Window<T, NX, NY>& w, T (&mf)[NX], T (&Pii)[NX][NX],
                         T (&PiL)[NX][NX]) {
  window_step<T, NX, NY, true>(M, w, 1, mf, Pii, PiL);
}
template <typename T, int NX, int NY>
SRTM_DEV void first_step(const TvModel<T, NX, NY>& M, int L, const Window<T, NX, NY>& w, T (&mf)[NX],
                         T (&Pii)[NX][NX], T (&PiL)[NX][NX]) {
  TvSteps<T, NX, NY> st;
  st.template next<true, false>(M, L, w, mf, Pii, PiL);
}

template <typename T, int NX, int NY>
SRTM_DEV void load_prior(const T* __restrict__ carry, const T* __restrict__ m0, const T* __restrict__ P0,
                         int64_t k, T (&m)[NX], T (&P)[NX][NX]) {
  constexpr int ST = NX + NX * NX;
  if (k == 0) {
    gloadv(m, m0);
    gload(P, P0);
  } else {
    gloadv(m, carry + (k - 1) * ST);
    gload(P, carry + (k - 1) * ST + NX);
  }
}

// ---------------------------------------------------------------- known inputs
// With x_t = A x_{t-1} + B u_{t-1} + w_{t-1} (eq. original-linear-SSM), window k's own
// inputs add the deterministic response z_{k,i} = A z_{k,i-1} + B u_{k,i-1}, z_{k,0} = 0, to
// its fast states given x_{k-1,l}: in eq. h-k-l-2 B_bar u_bar_k = z_{k,l}, and in eq. y-k-l-2
// D_bar u_bar_k = mu_k = (C/l) sum_i z_{k,i}. Hence the filter element's d gains z_{k,l}, every
// innovation uses y_k - mu_k, m^f_{k,i} gains z_{k,i}, and the smoother's prediction of
// x_{k+1,1} gains B u_{k+1,0}. No covariance depends on the inputs.

// B u of one fast step (uk: that step's nu inputs).
template <typename T, int NX>
SRTM_DEV void input_drive(const InputView<T>& in, const T* __restrict__ uk, T (&bu)[NX]) {
#pragma unroll
  for (int r = 0; r < NX; ++r) bu[r] = T(0);
#pragma unroll
  for (int j = 0; j < NU_MAX; ++j) {
    if (j < in.nu) {
      const T uj = gld(uk + j);
#pragma unroll
      for (int r = 0; r < NX; ++r) bu[r] = my_fma(gld(in.B + r * in.nu + j), uj, bu[r]);
    }
  }
}

// z <- A z + B u  (one fast step of the input response)
template <typename T, int NX>
SRTM_DEV void input_step(const InputView<T>& in, const T (&A)[NX][NX], const T* __restrict__ uk, T (&z)[NX]) {
  T nz[NX];
  input_drive(in, uk, nz);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int q = 0; q < NX; ++q) nz[r] = my_fma(A[r][q], z[q], nz[r]);
#pragma unroll
  for (int r = 0; r < NX; ++r) z[r] = nz[r];
}

// Input response of window k < N from its inputs: zL = z_{k,l} and yt = y_k - mu_k. The inputs
// of 8 fast steps are loaded together before they are used, so that their loads are in flight
// at once.
template <typename T, int NX, int NY>
SRTM_DEV void window_input_pass(const Model<T, NX, NY>& M, const T* __restrict__ y, int64_t k, int L,
                                T (&yt)[NY], T (&zL)[NX]) {
  constexpr int CH = 8;
  T A[NX][NX], zs[NX];
  load(A, M.cst + M.lay.A);
#pragma unroll
  for (int r = 0; r < NX; ++r) zs[r] = zL[r] = T(0);
  const int nu = M.in.nu;
  const T* uk = M.in.u + k * L * nu;
#pragma unroll 1
  for (int i0 = 0; i0 < L; i0 += CH) {
    T ub[CH][NU_MAX];
#pragma unroll
    for (int t = 0; t < CH; ++t)
#pragma unroll
      for (int j = 0; j < NU_MAX; ++j) ub[t][j] = (i0 + t < L && j < nu) ? gld(uk + (i0 + t) * nu + j) : T(0);
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      if (i0 + t < L) {
        T nz[NX];
#pragma unroll
        for (int r = 0; r < NX; ++r) {
          T a = T(0);
#pragma unroll
          for (int j = 0; j < NU_MAX; ++j)
            if (j < nu) a = my_fma(gld(M.in.B + r * nu + j), ub[t][j], a);
#pragma unroll
          for (int q = 0; q < NX; ++q) a = my_fma(A[r][q], zL[q], a);
          nz[r] = a;
        }
#pragma unroll
        for (int r = 0; r < NX; ++r) {
          zL[r] = nz[r];
          zs[r] += nz[r];
        }
      }
    }
  }
  const T inv_l = T(1) / T(L);
#pragma unroll
  for (int r = 0; r < NY; ++r) {
    T s = T(0);
#pragma unroll
    for (int c = 0; c < NX; ++c) s = my_fma(gld(M.in.H + r * NX + c), zs[c], s);
    yt[r] = gld(y + k * NY + r) - s * inv_l;
  }
}

// Window k's measurement (zero past the last window): y_k itself without inputs, and with inputs
// y_k - mu_k and z_{k,l} from the per-window record (zL = 0 without inputs).
template <bool INP, typename T, int NX, int NY>
SRTM_DEV void window_meas(const Model<T, NX, NY>& M, const T* __restrict__ y, int64_t k, int64_t N,
                          T (&yt)[NY], T (&zL)[NX]) {
  constexpr int RS = NX + NY;
#pragma unroll
  for (int r = 0; r < NX; ++r) zL[r] = T(0);
  if constexpr (INP) {
#pragma unroll
    for (int r = 0; r < NY; ++r) yt[r] = (k < N) ? gld(M.in.rec + k * RS + r) : T(0);
#pragma unroll
    for (int r = 0; r < NX; ++r) zL[r] = (k < N) ? gld(M.in.rec + k * RS + NY + r) : T(0);
  } else {
#pragma unroll
    for (int r = 0; r < NY; ++r) yt[r] = (k < N) ? gld(y + k * NY + r) : T(0);
  }
}

// Smoother element of window k (eq. parallel-ak-smoothing, transposed S_k):
//   P^- = A P^f_{k,l} A^T + Q,  E = P^f_{k,1,l} A^T (P^-)^{-1},  g = m^f_{k,1} - E A m^f_{k,l},
//   S = P^f_{k,1} - E A (P^f_{k,1,l})^T = P^f_{k,1} - E P^- E^T;   last window: (0, m^f_{N,1}, P^f_{N,1}).
// Also returns P^-, (P^-)^{-1} and the predicted mean A m^f_{k,l}, which the smoother correction
// reuses. (A, Qm) is the model of the step into x_{k+1,1}. With inputs, z1 = B u_{k,0} is added to
// m^f_{k,1} and bnext = B u_{k+1,0} to the prediction.
template <bool INP, typename T, int NX, int NY, class MV>
SRTM_DEV int smoother_element(const MV& M, int L, const Window<T, NX, NY>& w, bool last,
                              const T (&mL)[NX], const T (&PL)[NX][NX], const T (&z1)[NX], const T (&bnext)[NX],
                              const T (&A)[NX][NX], const T (&Qm)[NX][NX], SElem<T, NX>& el, T (&Pmi)[NX][NX],
                              T (&mpred)[NX], T (&Pm)[NX][NX]) {
  T mf1[NX], Pf11[NX][NX], Pf1L[NX][NX];
  first_step(M, L, w, mf1, Pf11, Pf1L);
  if constexpr (INP) {
#pragma unroll
    for (int r = 0; r < NX; ++r) mf1[r] += z1[r];
  }
  int flag = 0;
  if (last) {
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      el.g[r] = mf1[r];
      mpred[r] = T(0);
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        el.E[r][c] = T(0);
        el.S[r][c] = Pf11[r][c];
        Pmi[r][c] = T(0);
        Pm[r][c] = T(0);
      }
    }
    return 0;
  }
  sandwich(A, PL, Qm, Pm);
  if (!spd_inv(Pm, Pmi)) flag |= SRTM_INFO_PRED_SINGULAR;
  mv(A, mL, mpred);
  if constexpr (INP) {
#pragma unroll
    for (int r = 0; r < NX; ++r) mpred[r] += bnext[r];
  }
  T PA[NX][NX];  // P^f_{1,l} A^T, which is also E P^-
  mm_nt(Pf1L, A, PA);
  mm(PA, Pmi, el.E);
  T Em[NX];
  mv(el.E, mpred, Em);
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    el.g[r] = mf1[r] - Em[r];
#pragma unroll
    for (int c = r; c < NX; ++c) {  // S = P^f_{1,1} - E P^- E^T = P^f_{1,1} - (P^f_{1,l} A^T) E^T
      T s = Pf11[r][c];
#pragma unroll
      for (int k = 0; k < NX; ++k) s = my_fma(-PA[r][k], el.E[c][k], s);
      el.S[r][c] = s;
      el.S[c][r] = s;
    }
  }
  return flag;
}

// ============================================================================ forward
// Vector part of eq. op-filter for two runs of 2^p elements (level-p coefficients).
template <typename T, int NX>
SRTM_DEV void level_vec_combine_g(const T* __restrict__ G, const T (&di)[NX], const T (&ei)[NX], T (&dj)[NX],
                                  T (&ej)[NX]) {
  constexpr int NN = NX * NX;
  T G1[NX][NX], G2[NX][NX], G3[NX][NX], G4[NX][NX];
  load(G1, G);
  load(G2, G + NN);
  load(G3, G + 2 * NN);
  load(G4, G + 3 * NN);
  T nd[NX], ne[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T s = dj[r], t = ei[r];
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      s = my_fma(G1[r][k], di[k], s);
      s = my_fma(G2[r][k], ej[k], s);
      t = my_fma(G3[r][k], ej[k], t);
      t = my_fma(-G4[r][k], di[k], t);
    }
    nd[r] = s;
    ne[r] = t;
  }
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    dj[r] = nd[r];
    ej[r] = ne[r];
  }
}

// Vector part of eq. op-filter for two runs of 2^p elements (level-p coefficients G1..G4, which
// follow each other in a level record).
template <typename T, int NX>
SRTM_DEV void level_vec_combine(const T* __restrict__ lev, const ConstLayout& lay, const T (&di)[NX],
                                const T (&ei)[NX], T (&dj)[NX], T (&ej)[NX]) {
  level_vec_combine_g<T, NX>(lev + lay.o_G1, di, ei, dj, ej);
}

// In-place up-sweep over the vector parts of the tile's elements (slots 0..TILE-1); `G` holds the
// coefficient blocks G1..G4 of levels 0..LOG_TILE-1, 4 nx^2 scalars per level.
template <typename T, int NX>
SRTM_DEV void fwd_upsweep(const T* __restrict__ G, const Slots<T>& S, int tid) {
  constexpr int NN = NX * NX;
#pragma unroll 1
  for (int p = 0; p < LOG_TILE; ++p) {
    const int s = 1 << p;
    // Pair j (slots j 2^{p+1} + s - 1 and j 2^{p+1} + 2s - 1) goes to thread j, so that the active
    // threads fill the first waves: every active wave reads the level's coefficients from LDS,
    // and those broadcast reads, not the arithmetic, set the time of a level.
    if (tid < (TILE >> (p + 1))) {
      const int dst = (tid << (p + 1)) + 2 * s - 1;
      T di[NX], ei[NX], dj[NX], ej[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        di[r] = S.at(r, dst - s);
        ei[r] = S.at(NX + r, dst - s);
        dj[r] = S.at(r, dst);
        ej[r] = S.at(NX + r, dst);
      }
      level_vec_combine_g<T, NX>(G + p * 4 * NN, di, ei, dj, ej);
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        S.at(r, dst) = dj[r];
        S.at(NX + r, dst) = ej[r];
      }
    }
    __syncthreads();
  }
}

// Vector part (d, eta) of window k's filter element from its measurement yt (y_k - mu_k with
// inputs) and its input response zL = z_{k,l}.
template <bool INP, typename T, int NX, int NY>
SRTM_DEV void fwd_element(const Model<T, NX, NY>& M, const T (&yt)[NY], const T (&zL)[NX], T (&d)[NX],
                          T (&e)[NX]) {
  T K[NX][NY], He[NX][NY];
  load(K, M.cst + M.lay.K);
  load(He, M.cst + M.lay.Heta);
  mv(K, yt, d);
  mv(He, yt, e);
  if constexpr (INP) {
#pragma unroll
    for (int r = 0; r < NX; ++r) d[r] += zL[r];
  }
}

// K1: per-tile aggregate of the vector parts (d, eta) of the filter elements; the whole up-sweep
// tree (2 nx rows of TILE slots) goes to `utree` for the per-tile forward pass.
template <bool INP, typename T, int NX, int NY>
SRTM_DEV void fwd_reduce_body(const T* __restrict__ y, int64_t N, const T* __restrict__ cst, int L,
                              InputView<T> in, T* __restrict__ tagg, T* __restrict__ utree, int64_t tile) {
  constexpr int NN = NX * NX;
  extern __shared__ char smraw[];
  T* smem = reinterpret_cast<T*>(smraw);  // 2 nx TILE slots, then
  T* sG = smem + 2 * NX * TILE;           // G1..G4 of levels 0..LOG_TILE-1 (fwd_reduce_lds_bytes)
  const Model<T, NX, NY> M{cst, make_const_layout(NX, NY, L), in};
  const Slots<T> S{smem, TILE};
  const int tid = threadIdx.x;
  const int64_t k = tile * TILE + tid;
  // The level coefficients were written by an earlier launch, possibly on another die: one load
  // each, all in flight together, instead of a dependent round trip per level.
  for (int q = tid; q < LOG_TILE * 4 * NN; q += TILE) sG[q] = gld(M.level(q / (4 * NN)) + M.lay.o_G1 + q % (4 * NN));
  T yt[NY], zL[NX], d[NX], e[NX];
  if constexpr (INP) {  // one pass over the window's inputs; later kernels read the record
    if (k < N) {
      window_input_pass(M, y, k, L, yt, zL);
      constexpr int RS = NX + NY;
#pragma unroll
      for (int r = 0; r < NY; ++r) put_global(M.in.rec + k * RS + r, yt[r]);
#pragma unroll
      for (int r = 0; r < NX; ++r) put_global(M.in.rec + k * RS + NY + r, zL[r]);
    } else {
#pragma unroll
      for (int r = 0; r < NY; ++r) yt[r] = T(0);
#pragma unroll
      for (int r = 0; r < NX; ++r) zL[r] = T(0);
    }
  } else {
    window_meas<false>(M, y, k, N, yt, zL);
  }
  fwd_element<INP>(M, yt, zL, d, e);
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    S.at(r, tid) = d[r];
    S.at(NX + r, tid) = e[r];
  }
  __syncthreads();
  fwd_upsweep<T, NX>(sG, S, tid);
  T* ut = utree + tile * (2 * NX * TILE);
#pragma unroll
  for (int r = 0; r < 2 * NX; ++r) put_global(ut + r * TILE + tid, S.at(r, tid));
  if (tid == TILE - 1) {
#pragma unroll
    for (int r = 0; r < 2 * NX; ++r) tagg[tile * 2 * NX + r] = S.at(r, TILE - 1);
  }
}

// K2 (Kogge-Stone form): tile-level forward scan in one workgroup of KS threads. Thread tau
// holds the vector parts of its chunk of 2^lchunk tiles (matrices Theta(2^lchunk TILE)); the
// prior (m0, P0) is folded into thread 0, which makes it a state. At step q, threads in
// [2^q, 2^{q+1}) combine the state of thread tau - 2^q with their run (one state combine,
// eq. op-filter with F_i = 0) and become states; the others merge two runs of equal length
// with the shared level coefficients. Thread tau then walks its chunk from its exclusive
// state, writing each tile's incoming state.
template <typename T, int NX, int NY>
SRTM_DEV void fwd_tiles_body(const T* __restrict__ tagg, int64_t nt, int lchunk, int steps, int nlev,
                             const T* __restrict__ cst, int L, const T* __restrict__ m0, const T* __restrict__ P0,
                             T* __restrict__ tstate, int32_t* info) {
  constexpr int NN = NX * NX, ST = NX + NN;
  extern __shared__ char smraw[];
  const Slots<T> S{reinterpret_cast<T*>(smraw), KS};
  const Model<T, NX, NY> M{cst, make_const_layout(NX, NY, L)};
  const int tid = threadIdx.x;
  const int64_t c = int64_t(1) << lchunk;
  const int64_t t0 = tid * c;
  int flag = 0;
  const int l0 = LOG_TILE + lchunk;
  // The level records this scan uses (LOG_TILE .. nlev-1) are copied to LDS behind the slots
  // first, so that no step waits on a memory round trip for its coefficients.
  T* slev = reinterpret_cast<T*>(smraw) + KS * (NX + NN);
  {
    const T* gl = M.level(LOG_TILE);
    const int n = (nlev - LOG_TILE) * M.lay.lev_stride;
    for (int q = tid; q < n; q += KS) slev[q] = gld(gl + q);
  }
  auto level = [&](int p) { return slev + (p - LOG_TILE) * M.lay.lev_stride; };
  T d[NX], e[NX];
  T d0[NX], e0[NX];  // vector parts of tile t0 (c = 2), reused by the walk at the end
  if (c == 1) {
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      d[r] = (t0 < nt) ? gld(tagg + t0 * 2 * NX + r) : T(0);
      e[r] = (t0 < nt) ? gld(tagg + t0 * 2 * NX + NX + r) : T(0);
    }
  } else if (c == 2) {  // two runs of 2^LOG_TILE windows: vector parts only
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      d[r] = (t0 + 1 < nt) ? gld(tagg + (t0 + 1) * 2 * NX + r) : T(0);
      e[r] = (t0 + 1 < nt) ? gld(tagg + (t0 + 1) * 2 * NX + NX + r) : T(0);
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      d0[r] = (t0 < nt) ? gld(tagg + t0 * 2 * NX + r) : T(0);
      e0[r] = (t0 < nt) ? gld(tagg + t0 * 2 * NX + NX + r) : T(0);
    }
    __syncthreads();  // the level copy is complete
    level_vec_combine(level(LOG_TILE), M.lay, d0, e0, d, e);
  } else {  // fold the chunk with full combines (tiles past the end carry zero vectors)
    __syncthreads();  // the level copy is complete
    const T* lv = level(LOG_TILE);
    FElem<T, NX> acc, b;
    load(b.F, lv + M.lay.o_F);
    load(b.D, lv + M.lay.o_D);
    load(b.J, lv + M.lay.o_J);
#pragma unroll 1
    for (int64_t j = 0; j < c; ++j) {
      const int64_t t = t0 + j;
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        b.d[r] = (t < nt) ? tagg[t * 2 * NX + r] : T(0);
        b.e[r] = (t < nt) ? tagg[t * 2 * NX + NX + r] : T(0);
      }
      if (j == 0) {
        acc = b;
      } else if (!elem_combine(acc, b, acc)) {
        flag |= SRTM_INFO_COMBINE_SINGULAR;
      }
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      d[r] = acc.d[r];
      e[r] = acc.e[r];
    }
  }
  if (c == 1) __syncthreads();  // the level copy is complete
  T m[NX], P[NX][NX];
  if (tid == 0) {
    gloadv(m, m0);
    gload(P, P0);
    symmetrize(P);
    const T* lv = level(l0);
    T F[NX][NX], D[NX][NX], J[NX][NX];
    load(F, lv + M.lay.o_F);
    load(D, lv + M.lay.o_D);
    load(J, lv + M.lay.o_J);
    if (!state_combine(m, P, F, d, D, e, J)) flag |= SRTM_INFO_COMBINE_SINGULAR;
  }
  // While 2s < 64, wave 0 holds both the lanes [s, 2s) that form states and lanes [2s, 64) that
  // merge vector runs, and would run both combines one after the other. The vector runs of those
  // lanes are kept by lane tid - 64 of wave 1 instead (its second vector combine of the step):
  // the helper writes the run into the slot at the next step's start, and the owner reads it back
  // from there when it becomes a state. Barriers are unchanged.
  const bool helper = tid >= 64 && tid < 128;
  const int hl = tid - 64;  // the chunk a helper keeps
  T hd[NX], he[NX];         // its run
#pragma unroll 1
  for (int q = 0; q < steps; ++q) {
    const int s = 1 << q;
    const bool kept_prev = q >= 1 && s <= 32;  // the previous step kept the runs of [s, 64)
    const bool keep_now = 2 * s < 64;          // this step keeps the runs of [2s, 64)
    if (tid < s) {
      st_state<T, NX>(S, tid, m, P);
    } else if (!(tid < 64 && kept_prev)) {
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        S.at(r, tid) = d[r];
        S.at(NX + r, tid) = e[r];
      }
    }
    if (helper && kept_prev && hl >= s) {
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        S.at(r, hl) = hd[r];
        S.at(NX + r, hl) = he[r];
      }
    }
    __syncthreads();
    const bool gets_state = tid >= s && tid < 2 * s;
    const bool own_vec = tid >= 2 * s && !(tid < 64 && keep_now);
    const bool helps = helper && keep_now && hl >= 2 * s;
    T mo[NX], Po[NX][NX], dl[NX], el[NX], hdl[NX], hel[NX];
    if (gets_state) {
      ld_state<T, NX>(S, tid - s, mo, Po);
      if (tid < 64 && kept_prev) {  // the run its helper kept
#pragma unroll
        for (int r = 0; r < NX; ++r) {
          d[r] = S.at(r, tid);
          e[r] = S.at(NX + r, tid);
        }
      }
    } else if (own_vec) {
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        dl[r] = S.at(r, tid - s);
        el[r] = S.at(NX + r, tid - s);
      }
    }
    if (helps) {
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        hdl[r] = S.at(r, hl - s);
        hel[r] = S.at(NX + r, hl - s);
        if (q == 0) {  // the owner's own run, stored above
          hd[r] = S.at(r, hl);
          he[r] = S.at(NX + r, hl);
        }
      }
    }
    __syncthreads();
    const T* lv = level(l0 + q);
    if (gets_state) {
      T F[NX][NX], D[NX][NX], J[NX][NX];
      load(F, lv + M.lay.o_F);
      load(D, lv + M.lay.o_D);
      load(J, lv + M.lay.o_J);
      if (!state_combine(mo, Po, F, d, D, e, J)) flag |= SRTM_INFO_COMBINE_SINGULAR;
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        m[r] = mo[r];
#pragma unroll
        for (int cc = 0; cc < NX; ++cc) P[r][cc] = Po[r][cc];
      }
    } else if (own_vec) {
      level_vec_combine(lv, M.lay, dl, el, d, e);
    }
    if (helps) level_vec_combine(lv, M.lay, hdl, hel, hd, he);
  }
  // every active thread now holds the inclusive state through its chunk
  st_state<T, NX>(S, tid, m, P);
  __syncthreads();
  if (t0 < nt) {
    T X[NX], XP[NX][NX];
    if (tid == 0) {
      gloadv(X, m0);
      gload(XP, P0);
      symmetrize(XP);
    } else {
      ld_state<T, NX>(S, tid - 1, X, XP);
    }
    const T* lv = level(LOG_TILE);
    T F[NX][NX], D[NX][NX], J[NX][NX];
    load(F, lv + M.lay.o_F);
    load(D, lv + M.lay.o_D);
    load(J, lv + M.lay.o_J);
#pragma unroll 1
    for (int64_t t = t0; t < t0 + c && t < nt; ++t) {
#pragma unroll
      for (int r = 0; r < NX; ++r) tstate[t * ST + r] = X[r];
#pragma unroll
      for (int r = 0; r < NX; ++r)
#pragma unroll
        for (int cc = 0; cc < NX; ++cc) tstate[t * ST + NX + r * NX + cc] = XP[r][cc];
      if (t + 1 < t0 + c && t + 1 < nt) {
        T dt[NX], et[NX];
        if (c == 2) {
#pragma unroll
          for (int r = 0; r < NX; ++r) {
            dt[r] = d0[r];
            et[r] = e0[r];
          }
        } else {
          gloadv(dt, tagg + t * 2 * NX);
          gloadv(et, tagg + t * 2 * NX + NX);
        }
        if (!state_combine(X, XP, F, dt, D, et, J)) flag |= SRTM_INFO_COMBINE_SINGULAR;
      }
    }
  }
  if (flag && info) atomicOr(info, flag);
}

// K5: reverse tile-level scan in one workgroup of KS threads. Thread r holds the aggregate of
// its chunk of 2^lchunk consecutive tiles, counted from the end (thread 0 holds the last tiles),
// folded under eq. op-smoother (earlier (x) later), and merges it with all later runs (lane
// shuffles inside a wave, then the later waves' aggregates). Every run reaching the
// last window has E = 0, i.e. is the smoothed state at its first window; thread r then walks
// its chunk backwards from the state after it, writing per tile the smoothed state of the
// first window after the tile (zero after the last tile).
template <typename T, int NX>
SRTM_DEV void ld_selem_global(const T* __restrict__ src, SElem<T, NX>& x) {
  constexpr int NN = NX * NX;
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    x.g[i] = gld(src + NN + i);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      x.E[i][c] = gld(src + i * NX + c);
      x.S[i][c] = gld(src + NN + NX + i * NX + c);
    }
  }
}

template <typename T, int NX>
SRTM_DEV void selem_identity(SElem<T, NX>& x) {
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    x.g[i] = T(0);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      x.E[i][c] = (i == c) ? T(1) : T(0);
      x.S[i][c] = T(0);
    }
  }
}

template <typename T, int NX, int NY>
SRTM_DEV void bwd_tiles_body(const T* __restrict__ tagg, int64_t nt, int lchunk, int steps, T* __restrict__ tstate) {
  constexpr int NN = NX * NX, SE = 2 * NN + NX, ST = NX + NN;
  extern __shared__ char smraw[];
  const Slots<T> S{reinterpret_cast<T*>(smraw), KS};
  const int tid = threadIdx.x;
  const int64_t c = int64_t(1) << lchunk;
  const int64_t thi = nt - 1 - tid * c;  // the chunk is tiles thi - c + 1 .. thi (those >= 0)
  SElem<T, NX> x, xhi;  // xhi: the aggregate of tile thi itself (c = 2), reused by the walk
  if (thi >= 0 && c == 2) {  // both loads in flight together
    SElem<T, NX> a;
    ld_selem_global(tagg + thi * SE, xhi);
    if (thi - 1 >= 0) {
      ld_selem_global(tagg + (thi - 1) * SE, a);
      selem_combine(a, xhi, x);
    } else {
      x = xhi;
    }
  } else if (thi >= 0) {
    ld_selem_global(tagg + thi * SE, x);
#pragma unroll 1
    for (int64_t t = thi - 1; t > thi - c && t >= 0; --t) {
      SElem<T, NX> a;
      ld_selem_global(tagg + t * SE, a);
      selem_combine(a, x, x);
    }
  } else {
    selem_identity(x);
  }
  // Thread r ends with its run merged with every later run (threads r - 1 .. 0): within each
  // wave by lane shuffles (distances below 64), then each wave with the aggregates of the waves
  // before it (later tiles; lane 63 holds its wave's), through LDS.
  {
    const int lane = tid & 63, wv = tid >> 6;
    const int lim = steps < 6 ? steps : 6;
#pragma unroll 1
    for (int q = 0; q < lim; ++q) selem_merge_lane<false>(x, 1 << q, lane >= (1 << q));
    if (steps > 6) {
      if (lane == 63) st_selem(S, wv, x);
      __syncthreads();
#pragma unroll 1
      for (int v = wv - 1; v >= 0; --v) {  // x (x) A_{wv-1} (x) ... (x) A_0, left to right
        SElem<T, NX> a;
        ld_selem(S, v, a);
        selem_combine(x, a, x);
      }
      __syncthreads();  // the aggregates are read before the slots take the results
    }
  }
  st_selem(S, tid, x);
  __syncthreads();
  if (thi >= 0) {
    T m[NX], P[NX][NX];
    if (tid > 0) {
      SElem<T, NX> nxt;
      ld_selem(S, tid - 1, nxt);
#pragma unroll
      for (int i = 0; i < NX; ++i) {
        m[i] = nxt.g[i];
#pragma unroll
        for (int cc = 0; cc < NX; ++cc) P[i][cc] = nxt.S[i][cc];
      }
    } else {
#pragma unroll
      for (int i = 0; i < NX; ++i) {
        m[i] = T(0);
#pragma unroll
        for (int cc = 0; cc < NX; ++cc) P[i][cc] = T(0);
      }
    }
#pragma unroll 1
    for (int64_t t = thi; t > thi - c && t >= 0; --t) {
#pragma unroll
      for (int i = 0; i < NX; ++i) tstate[t * ST + i] = m[i];
#pragma unroll
      for (int i = 0; i < NX; ++i)
#pragma unroll
        for (int cc = 0; cc < NX; ++cc) tstate[t * ST + NX + i * NX + cc] = P[i][cc];
      if (t - 1 > thi - c && t - 1 >= 0) {
        if (c == 2) {
          sstate_combine(xhi, m, P);
        } else {
          SElem<T, NX> a;
          ld_selem_global(tagg + t * SE, a);
          sstate_combine(a, m, P);
        }
      }
    }
  }
}

// Output staging. Each lane computes one window's blocks; records are written to LDS
// and copied out by the whole wave so that consecutive lanes store consecutive 16-byte
// chunks. Covariance records (nx^2 scalars) are flushed every fast step; means are
// gathered over G consecutive fast steps so that a record fills whole cache lines.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
template <int CH> struct Chunk;
template <> struct Chunk<16> { using type = u32x4; };
template <> struct Chunk<8> { using type = u32x2; };
template <> struct Chunk<4> { using type = unsigned int; };

// Store of one output chunk. Outputs are written once and never read back by the library;
// when a flush writes whole 128-byte lines they are stored non-temporally (streamed past the
// L2), otherwise normally, so that partial lines can merge in the L2 first.
template <bool NT, typename V>
SRTM_DEV void put_chunk(char* p, const V& v) {
  using G = __attribute__((address_space(1))) V*;  // outputs are device memory: global stores
  if constexpr (NT)
    __builtin_nontemporal_store(v, (G)p);
  else
    *(G)p = v;
}


// Copies records w = 0..nvalid-1 (nvalid <= 64) of RB bytes (stride SB bytes in LDS) to
// dst + w * gstride bytes in chunks of CH bytes. A record is PER = RB / CH chunks; one store
// instruction moves WPI = 64 / PER whole records (lane l: chunk l mod PER of record
// l / PER + r WPI; the last 64 mod PER lanes idle), so every store address is a wave-uniform base
// plus one loop-invariant 32-bit lane offset.
template <int RB, int SB, int CH, bool NT>
SRTM_DEV void flush_chunks(int lane, int nvalid, const char* __restrict__ lds, char* __restrict__ dst,
                           int64_t gstride) {
  constexpr int PER = RB / CH;
  static_assert(RB % CH == 0 && SB % CH == 0 && PER <= 64, "whole chunks, at most one per lane");
  constexpr int WPI = 64 / PER;
  constexpr int NIT = (64 + WPI - 1) / WPI;
  using V = typename Chunk<CH>::type;
  const int wl = lane / PER, pl = lane - wl * PER;
  const unsigned int lo = (unsigned int)(wl * gstride) + (unsigned int)(pl * CH);
  const char* lsrc = lds + wl * SB + pl * CH;
  if constexpr (64 % PER == 0) {  // every lane busy: all LDS reads first, then the stores back to back
    V v[NIT];
#pragma unroll
    for (int r = 0; r < NIT; ++r) v[r] = *reinterpret_cast<const V*>(lsrc + r * WPI * SB);
    if (nvalid == 64) {
#pragma unroll
      for (int r = 0; r < NIT; ++r) put_chunk<NT>(dst + (int64_t)r * WPI * gstride + lo, v[r]);
    } else {
#pragma unroll
      for (int r = 0; r < NIT; ++r)
        if (wl + r * WPI < nvalid) put_chunk<NT>(dst + (int64_t)r * WPI * gstride + lo, v[r]);
    }
  } else {  // groups of four instructions (reads, then stores), to bound the registers held
    constexpr int G = 4;
    const bool act = wl < WPI;
#pragma unroll 1
    for (int r0 = 0; r0 < NIT; r0 += G) {
      V v[G];
#pragma unroll
      for (int j = 0; j < G; ++j)
        if (r0 + j < NIT && act && wl + (r0 + j) * WPI < 64)
          v[j] = *reinterpret_cast<const V*>(lsrc + (r0 + j) * WPI * SB);
#pragma unroll
      for (int j = 0; j < G; ++j)
        if (r0 + j < NIT && act && wl + (r0 + j) * WPI < nvalid)
          put_chunk<NT>(dst + (int64_t)(r0 + j) * WPI * gstride + lo, v[j]);
    }
  }
}

// Chunks of 16 bytes when the record length and LDS stride allow them and the destination and
// record stride are 16-byte aligned, 8 bytes for records that are 8- but not 16-byte multiples,
// 4-byte words otherwise. Without GENERAL only records that divide the wave (64 mod PER = 0) go
// in chunks. GENERAL (4-byte element types) also chunks the others, e.g. the 144-byte records of
// a 6 x 6 float covariance; the float64 recovery of the mixed-pair kernels, which spills heavily,
// returned wrong results for unchanged cases with it, so float64 keeps 4-byte words for them.
template <int RB, int SB, bool NT = false, bool GENERAL = false>
SRTM_DEV void flush_records(int lane, int nvalid, const char* __restrict__ lds, char* __restrict__ dst,
                            int64_t gstride) {
  const uintptr_t al = reinterpret_cast<uintptr_t>(dst) | (uintptr_t)gstride;
  if constexpr (RB % 16 == 0 && SB % 16 == 0 && RB / 16 <= 64 && (GENERAL || 64 % (RB / 16) == 0)) {
    if (al % 16 == 0) {
      flush_chunks<RB, SB, 16, NT>(lane, nvalid, lds, dst, gstride);
      return;
    }
  }
  if constexpr (RB % 16 != 0 && RB % 8 == 0 && SB % 8 == 0 && RB / 8 <= 64 && (GENERAL || 64 % (RB / 8) == 0)) {
    if (al % 8 == 0) {
      flush_chunks<RB, SB, 8, NT>(lane, nvalid, lds, dst, gstride);
      return;
    }
  }
  if constexpr (RB % 8 != 0 && 64 % (RB / 4) == 0) {  // whole records of 4-byte words per lane
    flush_chunks<RB, SB, 4, NT>(lane, nvalid, lds, dst, gstride);
    return;
  }
  for (int c = lane; c < nvalid * (RB / 4); c += 64) {  // 4-byte words
    const int w = c / (RB / 4), e = c - w * (RB / 4);
    put_global(reinterpret_cast<unsigned int*>(dst + w * gstride) + e,
               reinterpret_cast<const unsigned int*>(lds + w * SB)[e]);
  }
}

// Element-wise variant for a run-time record length (the last, partial group of means).
template <typename T>
SRTM_DEV void flush_records_rt(int lane, int nvalid, const char* __restrict__ lds, int SB, T* __restrict__ dst,
                               int64_t gstride_elems, int nel) {
  for (int c = lane; c < nvalid * nel; c += 64) {
    const int w = c / nel, e = c - w * nel;
    put_global(dst + w * gstride_elems + e, reinterpret_cast<const T*>(lds + w * SB)[e]);
  }
}

// Fast steps gathered into one output record: the largest power of two (at most 8) for
// which the record still fits in one 128-byte line.
constexpr int line_group(int bytes) {
  int g = 1;
  while (g < 8 && 2 * g * bytes <= 128) g *= 2;
  return g;
}

template <typename T, int NX>
struct OutStage {
  static constexpr int NN = NX * NX;
  static constexpr int GM = line_group(NX * (int)sizeof(T));   // means per record
  static constexpr int GP = line_group(NN * (int)sizeof(T));   // covariances per record
  static constexpr int RBM = GM * NX * (int)sizeof(T), RBP = GP * NN * (int)sizeof(T);
  static constexpr int SBP = ((RBP + 15) / 16) * 16 + 16;   // LDS bytes per lane (padded)
  static constexpr int SBM = ((RBM + 15) / 16) * 16 + 16;
  static constexpr int BYTES = 64 * (SBP + SBM);             // per wave
  char* pbuf;
  char* mbuf;
  SRTM_DEV OutStage(char* base) : pbuf(base), mbuf(base + 64 * SBP) {}
  // blocks of fast step i (1-based)
  SRTM_DEV void put(int lane, int i, const T (&m)[NX], const T (&P)[NX][NX]) const {
    T* pp = reinterpret_cast<T*>(pbuf + lane * SBP) + ((i - 1) % GP) * NN;
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NX; ++c) pp[r * NX + c] = P[r][c];
    T* mp = reinterpret_cast<T*>(mbuf + lane * SBM) + ((i - 1) % GM) * NX;
#pragma unroll
    for (int r = 0; r < NX; ++r) mp[r] = m[r];
  }
  // After put(i): flush the covariance and mean groups that step i completes. The record of
  // window w0 + w for fast steps i0 .. i0+g-1 starts at out[((w0 + w) L + i0 - 1) * size].
  SRTM_DEV void flush(int lane, int nvalid, T* m_out, T* P_out, int64_t w0, int L, int i, int ilim) const {
    const int sp = (i - 1) % GP, sm = (i - 1) % GM;
    if (P_out && (sp == GP - 1 || i == ilim)) {
      T* dst = P_out + (w0 * L + (i - sp - 1)) * NN;
      if (sp == GP - 1)
        flush_records<RBP, SBP, RBP % 128 == 0, sizeof(T) == 4>(lane, nvalid, pbuf, reinterpret_cast<char*>(dst),
                                                (int64_t)L * NN * sizeof(T));
      else
        flush_records_rt<T>(lane, nvalid, pbuf, SBP, dst, (int64_t)L * NN, (sp + 1) * NN);
    }
    if (m_out && (sm == GM - 1 || i == ilim)) {
      T* dst = m_out + (w0 * L + (i - sm - 1)) * NX;
      if (sm == GM - 1)
        flush_records<RBM, SBM, RBM % 128 == 0, sizeof(T) == 4>(lane, nvalid, mbuf, reinterpret_cast<char*>(dst),
                                                (int64_t)L * NX * sizeof(T));
      else
        flush_records_rt<T>(lane, nvalid, mbuf, SBM, dst, (int64_t)L * NX, (sm + 1) * NX);
    }
  }
  // slow-rate output: the blocks of fast step 1 (call right after put(1)), contiguous windows
  SRTM_DEV void flush_slow(int lane, int nvalid, T* m_out, T* P_out, int64_t w0) const {
    if (m_out)
      flush_records<NX * (int)sizeof(T), SBM, false, sizeof(T) == 4>(lane, nvalid, mbuf, reinterpret_cast<char*>(m_out + w0 * NX),
                                              (int64_t)NX * sizeof(T));
    if (P_out)
      flush_records<NN * (int)sizeof(T), SBP, false, sizeof(T) == 4>(lane, nvalid, pbuf, reinterpret_cast<char*>(P_out + w0 * NN),
                                              (int64_t)NN * sizeof(T));
  }
};

template <typename T, int NX>
SRTM_DEV bool finite_state(const T (&m)[NX], const T (&P)[NX][NX]) {
  bool ok = true;
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    ok = ok && isfinite(m[r]);
#pragma unroll
    for (int c = r; c < NX; ++c) ok = ok && isfinite(P[r][c]);
  }
  return ok;
}

// Per tile, every window's exclusive state (m^f_{k-1,l}, P^f_{k-1,l}) in (mprev, Pprev) and inclusive
// state (m^f_{k,l}, P^f_{k,l}) in (m, P). Window j of the tile is preceded inside the tile by the
// aligned runs of 2^p windows for the set bits p of j, and the tile's up-sweep tree holds the vector
// part of each such run [a, a + 2^p) in slot a + 2^p - 1 (no higher level of the in-place tree writes
// there); their matrix parts are the level records. So each lane folds, highest bit first, the
// tile's incoming state with those runs (eq. op-filter with the left operand a state) and then with
// its own element: the same combines as a tree down-sweep, with no exchange between lanes.
// S needs TILE * 2 nx scalars; (yt, zL): window k's measurement and input response (window_meas);
// `tree`: the tile's up-sweep tree as the tile reduction left it (2 nx rows of TILE slots).
// INCL false: the exclusive state only ((m, P) untouched).
template <bool INP, typename T, int NX, int NY, bool INCL = true>
SRTM_DEV int fwd_tile_states(const Model<T, NX, NY>& M, const Slots<T>& S, const T (&yt)[NY], const T (&zL)[NX],
                             int64_t k, const T* __restrict__ m0, const T* __restrict__ P0,
                             const T* __restrict__ tile_state, const T* __restrict__ tree, T (&mprev)[NX],
                             T (&Pprev)[NX][NX], T (&m)[NX], T (&P)[NX][NX]) {
  const int tid = threadIdx.x;
  int flag = 0;
#pragma unroll
  for (int r = 0; r < 2 * NX; ++r) S.at(r, tid) = gld(tree + r * TILE + tid);
  T d[NX], e[NX];  // the window's own element, for the inclusive state
  fwd_element<INP>(M, yt, zL, d, e);
  if (k == 0) {  // the prior itself
    gloadv(mprev, m0);
    gload(Pprev, P0);
  } else {
    gloadv(mprev, tile_state);
    gload(Pprev, tile_state + NX);
  }
  symmetrize(Pprev);
  __syncthreads();
#pragma unroll
  for (int p = LOG_TILE - 1; p >= 0; --p) {
    if ((tid >> p) & 1) {
      const int node = ((tid >> (p + 1)) << (p + 1)) + (1 << p) - 1;
      T dl[NX], el[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        dl[r] = S.at(r, node);
        el[r] = S.at(NX + r, node);
      }
      const T* lv = M.level(p);
      T F[NX][NX], D[NX][NX], J[NX][NX];
      load(F, lv + M.lay.o_F);
      load(D, lv + M.lay.o_D);
      load(J, lv + M.lay.o_J);
      if (!state_combine(mprev, Pprev, F, dl, D, el, J)) flag |= SRTM_INFO_COMBINE_SINGULAR;
    }
  }
  if constexpr (INCL) {  // exclusive state -> inclusive: X_k = X_{k-1} (x) a_k
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      m[r] = mprev[r];
#pragma unroll
      for (int c = 0; c < NX; ++c) P[r][c] = Pprev[r][c];
    }
    const T* lv = M.level(0);
    T F[NX][NX], D[NX][NX], J[NX][NX];
    load(F, lv + M.lay.o_F);
    load(D, lv + M.lay.o_D);
    load(J, lv + M.lay.o_J);
    if (!state_combine(m, P, F, d, D, e, J)) flag |= SRTM_INFO_COMBINE_SINGULAR;
  }
  return flag;
}

// Window k's filtered slow state (m^f_{k,l}, P^f_{k,l}) from its window quantities (window_setup
// on the exclusive state): the recovery's blocks at fast step l, m = A^l m' + c_l S^{-1} e (+ z_{k,l}
// with inputs) and P = A^l Y1 + Q_ll - c_l Y2 (upper triangle, mirrored). Equal to the inclusive
// combine X_{k-1} (x) a_k in exact arithmetic, at a fraction of its cost.
template <bool INP, typename T, int NX, int NY>
SRTM_DEV void window_slow_state(const Model<T, NX, NY>& M, int L, const Window<T, NX, NY>& w, const T (&zL)[NX],
                                T (&m)[NX], T (&P)[NX][NX]) {
  T AL[NX][NX], cL[NX][NY];
  M.get(AL, M.AL_off(L));
  M.get(cL, M.cL_off(L));
  const int oq = M.per_i_off(L) + M.lay.o_Qii;
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    T t = INP ? zL[r] : T(0);
#pragma unroll
    for (int k = 0; k < NX; ++k) t = my_fma(AL[r][k], w.mp[k], t);
#pragma unroll
    for (int k = 0; k < NY; ++k) t = my_fma(cL[r][k], w.Se[k], t);
    m[r] = t;
  }
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = r; c < NX; ++c) {
      T t = M.at(oq + r * NX + c);
#pragma unroll
      for (int k = 0; k < NX; ++k) t = my_fma(AL[r][k], w.Y1[k][c], t);
#pragma unroll
      for (int k = 0; k < NY; ++k) t = my_fma(-cL[r][k], w.Y2[k][c], t);
      P[r][c] = t;
      P[c][r] = t;
    }
}

// Writes the slow-rate carry (m^f_{k,l}, P^f_{k,l}) and, when requested, the slow-rate
// filter outputs of window k < N.
template <typename T, int NX>
SRTM_DEV int store_carry(int64_t k, const T (&m)[NX], const T (&P)[NX][NX], T* __restrict__ carry,
                         T* __restrict__ m_slow, T* __restrict__ P_slow) {
  constexpr int NN = NX * NX, ST = NX + NN;
#pragma unroll
  for (int r = 0; r < NX; ++r) put_global(carry + k * ST + r, m[r]);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) put_global(carry + k * ST + NX + r * NX + c, P[r][c]);
  if (m_slow) {
#pragma unroll
    for (int r = 0; r < NX; ++r) put_global(m_slow + k * NX + r, m[r]);
  }
  if (P_slow) {
#pragma unroll
    for (int r = 0; r < NN; ++r) put_global(P_slow + k * NN + r, P[r / NX][r % NX]);
  }
  return finite_state(m, P) ? 0 : SRTM_INFO_NONFINITE;
}

// K3 (filter only): per tile, the slow-rate carry and the slow-rate filter outputs.
template <bool INP, typename T, int NX, int NY>
SRTM_DEV void fwd_final_body(const T* __restrict__ y, int64_t N, int L, const T* __restrict__ cst, InputView<T> in,
                             const T* __restrict__ m0, const T* __restrict__ P0, const T* __restrict__ tstate,
                             const T* __restrict__ utree, T* __restrict__ carry, T* __restrict__ m_slow, T* __restrict__ P_slow, int32_t* info,
                             int64_t tile) {
  constexpr int ST = NX + NX * NX;
  extern __shared__ char smraw[];
  const Model<T, NX, NY> M{cst, make_const_layout(NX, NY, L), in};
  const Slots<T> S{reinterpret_cast<T*>(smraw), TILE};
  const int64_t k = tile * TILE + threadIdx.x;
  T yt[NY], zL[NX];
  window_meas<INP>(M, y, k, N, yt, zL);
  T mprev[NX], Pprev[NX][NX], m[NX], P[NX][NX];
  int flag = fwd_tile_states<INP>(M, S, yt, zL, k, m0, P0, tstate + tile * ST, utree + tile * (2 * NX * TILE), mprev,
                                  Pprev, m, P);
  if (k < N) flag |= store_carry(k, m, P, carry, m_slow, P_slow);
  if (flag && info) atomicOr(info, flag);
}

// ============================================================================ backward
// The smoother half of the fused forward/backward kernel for window k of tile `tile`, given the
// window quantities w (window_setup on the exclusive filter state), the inclusive filter state
// (m, P) and (An, Qn), the model of the step into x_{k+1,1}: its smoother element (eq.
// parallel-ak-smoothing), the in-tile reverse Kogge-Stone scan under eq. op-smoother, the tile
// aggregate and the per-window correction record (see fwd_bwd_body). Returns numerical status bits.
template <bool INP, typename T, int NX, int NY, class MV>
SRTM_DEV int smoother_part(const MV& M, const Slots<T>& S, int L, int64_t k, int64_t N,
                           const Window<T, NX, NY>& w, const T (&m)[NX], const T (&P)[NX][NX],
                           const T (&An)[NX][NX], const T (&Qn)[NX][NX], T* __restrict__ btagg,
                           T* __restrict__ sfx, int64_t tile) {
  constexpr int NN = NX * NX, SE = 2 * NN + NX, SF = sfx_stride(NX);
  const int tid = threadIdx.x;
  const bool valid = k < N;
  int flag = 0;
  SElem<T, NX> x;
  T B[NX][NX], Bm[NX], BPB[NX][NX];  // B = (P^-)^{-1} A, B^T (predicted mean), B^T P^- B = A^T B
  {
    T z1[NX], bnext[NX];  // B u_{k,0} and B u_{k+1,0}
#pragma unroll
    for (int r = 0; r < NX; ++r) z1[r] = bnext[r] = T(0);
    if constexpr (INP) {
      if (valid) input_drive(M.in, M.in.u + k * L * M.in.nu, z1);
      if (k + 1 < N) input_drive(M.in, M.in.u + (k + 1) * L * M.in.nu, bnext);
    }
    T Pmi[NX][NX], mpred[NX], Pm[NX][NX];
    const int f = smoother_element<INP>(M, L, w, k == N - 1, m, P, z1, bnext, An, Qn, x, Pmi, mpred, Pm);
    if (valid) flag |= f;
    mm(Pmi, An, B);
    mtv(B, mpred, Bm);
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = r; c < NX; ++c) {
        T t = T(0);
#pragma unroll
        for (int q = 0; q < NX; ++q) t = my_fma(An[q][r], B[q][c], t);
        BPB[r][c] = t;
        BPB[c][r] = t;
      }
  }
  if (!valid) {  // past the last window: a zero element (finite, and absorbed by E_N = 0)
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      x.g[r] = T(0);
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        x.E[r][c] = T(0);
        x.S[r][c] = T(0);
      }
    }
  }
  // Lane j ends with a_j (x) a_{j+1} (x) ... (x) a_{TILE-1}. Within each wave first, by lane
  // shuffles at distances 1 .. 32: lane l then holds its wave's elements l .. 63 merged, and lane
  // 0 the whole wave's. Then each wave merges with the aggregates of the waves after it, which
  // pass through LDS (runs of any length merge: eq. op-smoother carries whole matrices).
  {
    const int lane = tid & 63, wv = tid >> 6;
    constexpr int NW = TILE / 64;
#pragma unroll 1
    for (int s = 1; s < 64; s *= 2) selem_merge_lane<true>(x, s, lane + s < 64);
    __syncthreads();  // the slots switch from forward states to smoother elements
    if (lane == 0) st_selem(S, wv, x);
    __syncthreads();
#pragma unroll 1
    for (int v = wv + 1; v < NW; ++v) {  // x (x) A_{wv+1} (x) ... (x) A_{NW-1}, left to right
      SElem<T, NX> a;
      ld_selem(S, v, a);
      selem_combine(x, a, x);
    }
    __syncthreads();  // the aggregates are read before the slots take the suffixes
  }
  st_selem(S, tid, x);
  __syncthreads();
  if (tid == 0) {
    T* dst = btagg + tile * SE;
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      dst[NN + r] = x.g[r];
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        dst[r * NX + c] = x.E[r][c];
        dst[NN + NX + r * NX + c] = x.S[r][c];
      }
    }
  }
  SElem<T, NX> nxt;  // exclusive suffix; the identity (I, 0, 0) for the tile's last lane
  if (tid + 1 < TILE) {
    ld_selem(S, tid + 1, nxt);
  } else {
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      nxt.g[r] = T(0);
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        nxt.E[r][c] = (r == c) ? T(1) : T(0);
        nxt.S[r][c] = T(0);
      }
    }
  }
  if (valid) {
    T rec[SF];
    if (k < N - 1) {
      T SB[NX][NX];
      mm(nxt.S, B, SB);
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        T t = -Bm[r];
#pragma unroll
        for (int q = 0; q < NX; ++q) t = my_fma(B[q][r], nxt.g[q], t);
        rec[NN + r] = t;
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          T e = T(0);
#pragma unroll
          for (int q = 0; q < NX; ++q) e = my_fma(B[q][r], nxt.E[q][c], e);
          rec[r * NX + c] = e;
        }
      }
      int o = NN + NX;
#pragma unroll
      for (int r = 0; r < NX; ++r)
#pragma unroll
        for (int c = r; c < NX; ++c) {
          T t = -BPB[r][c];
#pragma unroll
          for (int q = 0; q < NX; ++q) t = my_fma(B[q][r], SB[q][c], t);
          rec[o++] = t;
        }
    } else {
#pragma unroll
      for (int r = 0; r < SF; ++r) rec[r] = T(0);
    }
    T* dst = sfx + k * SF;
#pragma unroll
    for (int r = 0; r < SF; ++r) put_global(dst + r, rec[r]);
  }
  return flag;
}

// K3s (smoother): per tile, the forward down-sweep of K3; then, from the exclusive and
// inclusive filter states of window k, its smoother element (eq. parallel-ak-smoothing), an
// in-tile reverse Kogge-Stone scan of those elements under eq. op-smoother, the tile's
// aggregate a_first (x) ... (x) a_last, and per window the smoother correction of eq.
// seq-smoothing-all written as terms linear in the smoothed state (m_in, P_in) that enters
// the tile from the right (the first window after it). With B = (P^-)^{-1} A and the
// in-tile exclusive suffix (E', g', S') = a_{k+1} (x) ... (x) a_{last of tile}:
//   v = A^T (P^-)^{-1} (m^s_{k+1,1} - A m^f_{k,l}) = Et m_in + gt,
//   W = A^T (P^-)^{-1} (P^s_{k+1,1} - P^-) (P^-)^{-1} A = Et P_in Et^T + St,
//   Et = B^T E',  gt = B^T (g' - A m^f_{k,l}),  St = B^T (S' - P^-) B;
// all three are zero for the last window, whose smoothed blocks equal the filtered ones.
template <bool INP, typename T, int NX, int NY>
SRTM_DEV void fwd_bwd_body(const T* __restrict__ y, int64_t N, int L, const T* __restrict__ cst, InputView<T> in,
                           const T* __restrict__ m0, const T* __restrict__ P0, const T* __restrict__ ftstate,
                           const T* __restrict__ utree, T* __restrict__ carry, T* __restrict__ m_slow, T* __restrict__ P_slow,
                           T* __restrict__ btagg, T* __restrict__ sfx, int32_t* info, int64_t tile) {
  constexpr int NN = NX * NX, ST = NX + NN, SE = 2 * NN + NX, SF = sfx_stride(NX);
  extern __shared__ char smraw[];
  const Model<T, NX, NY> M{cst, make_const_layout(NX, NY, L), in};
  const Slots<T> S{reinterpret_cast<T*>(smraw), TILE};
  const int tid = threadIdx.x;
  const int64_t k = tile * TILE + tid;
  const bool valid = k < N;
  T yt[NY], zL[NX];
  window_meas<INP>(M, y, k, N, yt, zL);
  T mprev[NX], Pprev[NX][NX], m[NX], P[NX][NX];
  int flag = fwd_tile_states<INP, T, NX, NY, false>(M, S, yt, zL, k, m0, P0, ftstate + tile * ST,
                                                    utree + tile * (2 * NX * TILE), mprev, Pprev, m, P);
  // The smoother element needs the window quantities of the exclusive state; the inclusive state
  // (the carry) follows from them.
  Window<T, NX, NY> w;
  if (!window_setup(M, L, mprev, Pprev, yt, w) && valid) flag |= SRTM_INFO_INNOVATION_NOT_PD;
  window_slow_state<INP>(M, L, w, zL, m, P);
  if (valid) flag |= store_carry(k, m, P, carry, m_slow, P_slow);

  T An[NX][NX], Qn[NX][NX];  // time-invariant: the step into x_{k+1,1} has the model's A and Q
  load(An, M.cst + M.lay.A);
  load(Qn, M.cst + M.lay.Q);
  flag |= smoother_part<INP>(M, S, L, k, N, w, m, P, An, Qn, btagg, sfx, tile);
  if (flag && info) atomicOr(info, flag);
}

// Per-window models in the recovery: the tile's A, Q and C (the caller's per-window F, Q, H)
// copied to LDS window-minor, entry j of window w at mdl[(j * TV_MS) + w] (j < nx^2: A, then Q,
// then C), with a padded column count so that the row-major reads of the copy spread over the
// banks. Windows past the end of the sequence get zeros.
constexpr int TV_MS = TILE + 1;
template <typename T, int NX, int NY>
constexpr size_t tv_model_lds_bytes() { return sizeof(T) * (size_t)(2 * NX * NX + NY * NX) * TV_MS; }

template <typename T, int NX, int NY>
SRTM_DEV void tv_model_to_lds(const T* __restrict__ Fa, const T* __restrict__ Qa, const T* __restrict__ Ha,
                              int64_t t0, int nw, T* mdl) {
  constexpr int NN = NX * NX, NXY = NX * NY;
  for (int q = threadIdx.x; q < TILE * NN; q += TILE) {
    const int w = q / NN, j = q % NN;
    mdl[j * TV_MS + w] = (w < nw) ? gld(Fa + t0 * NN + q) : T(0);
    mdl[(NN + j) * TV_MS + w] = (w < nw) ? gld(Qa + t0 * NN + q) : T(0);
  }
  for (int q = threadIdx.x; q < TILE * NXY; q += TILE) {
    const int w = q / NXY, j = q % NXY;
    mdl[(2 * NN + j) * TV_MS + w] = (w < nw) ? gld(Ha + t0 * NXY + q) : T(0);
  }
}

// The model view of window k: the call's constants block, or (TV) the window's own block with
// its A, Q and C from the tile's LDS copy `mdl` (per-window models: `cst` holds the blocks).
template <bool TV, typename T, int NX, int NY>
SRTM_DEV auto recover_model(const T* __restrict__ cst, int L, const InputView<T>& in, const T* mdl, int64_t k) {
  if constexpr (TV) {
    constexpr int NN = NX * NX;
    const int w = (int)(k % TILE);
    return TvModel<T, NX, NY, true>{tv_tile_base(cst, k, tv_block_size(NX, NY, L)), make_tv_layout(NX, NY, L), w,
                                    mdl + w, mdl + NN * TV_MS + w, mdl + 2 * NN * TV_MS + w, TV_MS};
  } else {
    return Model<T, NX, NY>{cst, make_const_layout(NX, NY, L), in};
  }
}

struct NoSteps {};

// Fast steps whose tables the time-invariant recovery holds in LDS at a time.
constexpr int RSTEPS = 32;

// K7: fast-rate recovery, one window per lane and a loop over the window's fast steps.
// MODE bit 1: filter blocks p(x_{k,i} | y_{1:k}); bit 2: smoothed blocks p(x_{k,i} | y_{1:N})
// (and the smoother's slow state, block i = 1) from the correction (v, W) that K3s left as
// terms linear in the smoothed state entering the tile; a workgroup covers exactly one tile.
// `ilim` is L when fast-rate outputs are requested and 1 when only the slow smoothed state is.
// TV: per-window model; `cst` then holds the per-window constants blocks (stored by tv_column)
// and Fa, Qa (with in.H) the per-window F, Q and H.
template <typename T, int NX, int NY, int MODE, bool INP, bool TV = false>
SRTM_DEV void recover_body(const T* __restrict__ y, int64_t N, int L, int ilim, const T* __restrict__ cst,
                           InputView<T> in, const T* __restrict__ Fa, const T* __restrict__ Qa,
                           const T* __restrict__ m0, const T* __restrict__ P0, const T* __restrict__ carry,
                           const T* __restrict__ sfx, const T* __restrict__ tin, T* __restrict__ mf_fast,
                           T* __restrict__ Pf_fast, T* __restrict__ ms_fast, T* __restrict__ Ps_fast,
                           T* __restrict__ ms_slow, T* __restrict__ Ps_slow, int32_t* info, int64_t tile) {
  constexpr int NN = NX * NX, ST = NX + NN, SF = sfx_stride(NX);
  static_assert(TILE == 256, "one recovery workgroup per tile");
  constexpr bool FILT = (MODE & 1) != 0, SMOOTH = (MODE & 2) != 0;
  static_assert(!(TV && FILT && SMOOTH), "per-window models: filter and smoother outputs in two passes "
                                         "(the LDS copy of the model follows one staging buffer per wave)");
  using Stg = OutStage<T, NX>;
  extern __shared__ char smraw[];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t k = tile * TILE + tid;
  const int64_t w0 = tile * TILE + wv * 64;
  const int nvalid = (int)((N - w0) < 64 ? ((N - w0) > 0 ? (N - w0) : 0) : 64);
  const Stg fst(smraw + (size_t)wv * Stg::BYTES * (FILT && SMOOTH ? 2 : 1));
  const Stg sst(smraw + (size_t)wv * Stg::BYTES * (FILT && SMOOTH ? 2 : 1) + (FILT && SMOOTH ? Stg::BYTES : 0));
  const bool valid = k < N;
  const int64_t kc = valid ? k : 0;   // clamped index for loads of padding lanes
  T* mdl = reinterpret_cast<T*>(smraw + (size_t)4 * Stg::BYTES * (FILT && SMOOTH ? 2 : 1));
  if constexpr (TV) {
    const int64_t t0 = tile * TILE;
    tv_model_to_lds<T, NX, NY>(Fa, Qa, in.H, t0, (int)((N - t0) < TILE ? (N - t0) : TILE), mdl);
    __syncthreads();
  }
  const auto M = recover_model<TV, T, NX, NY>(cst, L, in, mdl, k);
  T m[NX], P[NX][NX], yk[NY];
  load_prior<T, NX, NY>(carry, m0, P0, kc, m, P);
  if constexpr (INP) {
    T zL[NX];
    window_meas<true>(M, y, kc, N, yk, zL);
  } else {
    gloadv(yk, y + kc * NY);
  }
  Window<T, NX, NY> w;
  int flag = 0;
  if (!window_setup(M, L, m, P, yk, w) && valid) flag |= SRTM_INFO_INNOVATION_NOT_PD;
  T z[NX], un[NU_MAX];  // input response z_{k,i} and the next step's inputs (inputs only)
#pragma unroll
  for (int r = 0; r < NX; ++r) z[r] = T(0);
  const T* uk = INP ? in.u + kc * L * in.nu : nullptr;
  if constexpr (INP) {
#pragma unroll
    for (int j = 0; j < NU_MAX; ++j) un[j] = (j < in.nu) ? gld(uk + j) : T(0);
  }
  T v[NX], W[NX][NX];
  if (SMOOTH) {  // v = Et m_in + gt,  W = Et P_in Et^T + St
    const T* src = sfx + kc * SF;
    const T* ti = tin + tile * ST;
    T Et[NX][NX], mi[NX], Pi[NX][NX], EP[NX][NX];
    gload(Et, src);
    gloadv(mi, ti);
    gload(Pi, ti + NX);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      T t = gld(src + NN + r);
#pragma unroll
      for (int q = 0; q < NX; ++q) t = my_fma(Et[r][q], mi[q], t);
      v[r] = t;
    }
    mm(Et, Pi, EP);
    int o = NN + NX;
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = r; c < NX; ++c) {
        T t = gld(src + o++);
#pragma unroll
        for (int q = 0; q < NX; ++q) t = my_fma(EP[r][q], Et[c][q], t);
        W[r][c] = t;
        W[c][r] = t;
      }
  }
  bool fin = true;
  std::conditional_t<TV, TvSteps<T, NX, NY>, NoSteps> steps;
#pragma unroll 1
  for (int i = 1; i <= ilim; ++i) {
    T mf[NX], Pii[NX][NX], PiL[NX][NX];
    if constexpr (!TV) {
      // The per-step tables go to LDS, RSTEPS steps at a time: read per step as wave-uniform
      // scalar loads they outgrow the scalar registers (spilled to vector-register lanes and
      // read back every step).
      if ((i - 1) % RSTEPS == 0) {
        const int n = (ilim - i + 1 < RSTEPS ? ilim - i + 1 : RSTEPS) * M.lay.per_i_stride;
        const T* src = M.per_i(i);
        __syncthreads();  // every wave is done with the previous steps' tables
        staged_copy<8, T>(n, tid, TILE, [&](int q) { return gld(src + q); }, [&](int q, T v) { mdl[q] = v; });
        __syncthreads();
      }
    }
    if constexpr (TV) {
      steps.template next<SMOOTH, true>(M, L, w, mf, Pii, PiL);
    } else {  // step i's A^i, c_i, Q_ii and Q_il from the LDS copy
      const T* ps = mdl + ((i - 1) % RSTEPS) * M.lay.per_i_stride;
      T Ai[NX][NX], ci[NX][NY];
      load(Ai, ps + M.lay.o_Ai);
      load(ci, ps + M.lay.o_ci);
      step_blocks<SMOOTH>(
          w, Ai, ci, [&](int r, int c) { return ps[M.lay.o_Qii + r * NX + c]; },
          [&](int r, int c) { return ps[M.lay.o_QiL + r * NX + c]; }, mf, Pii, PiL);
    }
    if constexpr (INP) {  // z_i = A z_{i-1} + B u_{k,i-1}, the loads of step i+1 issued first
      T uc[NU_MAX];
#pragma unroll
      for (int j = 0; j < NU_MAX; ++j) {
        uc[j] = un[j];
        un[j] = (j < M.in.nu && i < L) ? gld(uk + i * M.in.nu + j) : T(0);
      }
      T A[NX][NX], nz[NX];
      load(A, M.cst + M.lay.A);
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        T t = T(0);
#pragma unroll
        for (int j = 0; j < NU_MAX; ++j)
          if (j < M.in.nu) t = my_fma(gld(M.in.B + r * M.in.nu + j), uc[j], t);
#pragma unroll
        for (int q = 0; q < NX; ++q) t = my_fma(A[r][q], z[q], t);
        nz[r] = t;
      }
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        z[r] = nz[r];
        mf[r] += z[r];
      }
    }
    if (FILT) {
      fin = fin && finite_state(mf, Pii);
      fst.put(lane, i, mf, Pii);
    }
    if (SMOOTH) {
      T ms[NX], Ps[NX][NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        T s = mf[r];
#pragma unroll
        for (int q = 0; q < NX; ++q) s = my_fma(PiL[r][q], v[q], s);
        ms[r] = s;
        T TW[NX];
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          T t = T(0);
#pragma unroll
          for (int q = 0; q < NX; ++q) t = my_fma(PiL[r][q], symget(W, q, c), t);
          TW[c] = t;
        }
#pragma unroll
        for (int c = r; c < NX; ++c) {
          T t = Pii[r][c];
#pragma unroll
          for (int q = 0; q < NX; ++q) t = my_fma(TW[q], PiL[c][q], t);
          Ps[r][c] = t;
          Ps[c][r] = t;
        }
      }
      fin = fin && finite_state(ms, Ps);
      sst.put(lane, i, ms, Ps);
    }
    wave_sync();
    if (FILT) fst.flush(lane, nvalid, mf_fast, Pf_fast, w0, L, i, ilim);
    if (SMOOTH) {
      if (i == 1) sst.flush_slow(lane, nvalid, ms_slow, Ps_slow, w0);
      sst.flush(lane, nvalid, ms_fast, Ps_fast, w0, L, i, ilim);
    }
    wave_sync();
  }
  if (!fin && valid) flag |= SRTM_INFO_NONFINITE;
  if (flag && info) atomicOr(info, flag);
}

// ============================================================================ sequential comparator
// The sequential route of Sec. III on the GPU, one lane per sequence and no scan: the IMKF walks
// the windows forwards (eq. prediction and eq. m-h-k-l, written as block l of the window filter
// of eq. update-fast) and stores the slow-rate carry (m^f_{k,l}, P^f_{k,l}); the sequential SRTM
// smoother then walks them backwards (eq. smoothing-dynamic, eq. seq-smoothing-all): with the
// smoothed state (m^s_{k+1,1}, P^s_{k+1,1}) of the window after, P^- = A P^f_{k,l} A^T + Q and
// B = (P^-)^{-1} A, the correction v = B^T (m^s_{k+1,1} - A m^f_{k,l}), W = B^T (P^s_{k+1,1} - P^-) B
// gives every fast step's smoothed blocks m^s_{k,i} = m^f_{k,i} + P^f_{k,i,l} v and
// P^s_{k,i} = P^f_{k,i,i} + P^f_{k,i,l} W P^f_{k,i,l}^T, and block i = 1 is the state the window before
// needs (eq. seq-smoothing-1). The per-window arithmetic is the parallel path's; only the order
// of evaluation differs (a recursion instead of the two scans). This is the paper's sequential
// comparison method (Sec. V), run on the same GPU.
template <typename T, int NX, int NY>
SRTM_DEV void seq_body(const T* __restrict__ y, int64_t N, int L, const T* __restrict__ cst,
                       const T* __restrict__ m0, const T* __restrict__ P0, T* __restrict__ carry,
                       T* __restrict__ ms_fast, T* __restrict__ Ps_fast, T* __restrict__ ms_slow,
                       T* __restrict__ Ps_slow, int32_t* info) {
  constexpr int NN = NX * NX, ST = NX + NN;
  const Model<T, NX, NY> M{cst, make_const_layout(NX, NY, L)};
  int flag = 0;
  bool fin = true;
  T m[NX], P[NX][NX];
  gloadv(m, m0);
  gload(P, P0);
  symmetrize(P);
#pragma unroll 1
  for (int64_t k = 0; k < N; ++k) {  // forward: the IMKF
    T yk[NY];
    gloadv(yk, y + k * NY);
    Window<T, NX, NY> w;
    if (!window_setup(M, L, m, P, yk, w)) flag |= SRTM_INFO_INNOVATION_NOT_PD;
    T PiL[NX][NX];
    window_step<T, NX, NY, false>(M, w, L, m, P, PiL);
#pragma unroll
    for (int r = 0; r < NX; ++r) put_global(carry + k * ST + r, m[r]);
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NX; ++c) put_global(carry + k * ST + NX + r * NX + c, P[r][c]);
  }
  T A[NX][NX], Qm[NX][NX];
  load(A, M.cst + M.lay.A);
  load(Qm, M.cst + M.lay.Q);
  T ms1[NX], Ps1[NX][NX];
#pragma unroll 1
  for (int64_t k = N - 1; k >= 0; --k) {  // backward: the sequential smoother
    T yk[NY];
    gloadv(yk, y + k * NY);
    if (k == 0) {
      gloadv(m, m0);
      gload(P, P0);
      symmetrize(P);
    } else {
      gloadv(m, carry + (k - 1) * ST);
      gload(P, carry + (k - 1) * ST + NX);
    }
    Window<T, NX, NY> w;
    if (!window_setup(M, L, m, P, yk, w)) flag |= SRTM_INFO_INNOVATION_NOT_PD;
    T v[NX], W[NX][NX];
    if (k == N - 1) {
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        v[r] = T(0);
#pragma unroll
        for (int c = 0; c < NX; ++c) W[r][c] = T(0);
      }
    } else {
      T mL[NX], PL[NX][NX], Pm[NX][NX], Pmi[NX][NX], B[NX][NX], d[NX], D[NX][NX], DB[NX][NX];
      gloadv(mL, carry + k * ST);
      gload(PL, carry + k * ST + NX);
      sandwich(A, PL, Qm, Pm);
      if (!spd_inv(Pm, Pmi)) flag |= SRTM_INFO_PRED_SINGULAR;
      mm(Pmi, A, B);
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        T t = ms1[r];
#pragma unroll
        for (int q = 0; q < NX; ++q) t = my_fma(-A[r][q], mL[q], t);
        d[r] = t;
#pragma unroll
        for (int c = 0; c < NX; ++c) D[r][c] = Ps1[r][c] - Pm[r][c];
      }
      mtv(B, d, v);
      mm(D, B, DB);
#pragma unroll
      for (int r = 0; r < NX; ++r)
#pragma unroll
        for (int c = r; c < NX; ++c) {
          T t = T(0);
#pragma unroll
          for (int q = 0; q < NX; ++q) t = my_fma(B[q][r], DB[q][c], t);
          W[r][c] = t;
          W[c][r] = t;
        }
    }
#pragma unroll 1
    for (int i = 1; i <= L; ++i) {
      T mf[NX], Pii[NX][NX], PiL[NX][NX], ms[NX], Ps[NX][NX];
      window_step<T, NX, NY, true>(M, w, i, mf, Pii, PiL);
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        T s = mf[r];
#pragma unroll
        for (int q = 0; q < NX; ++q) s = my_fma(PiL[r][q], v[q], s);
        ms[r] = s;
        T TW[NX];
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          T t = T(0);
#pragma unroll
          for (int q = 0; q < NX; ++q) t = my_fma(PiL[r][q], W[q][c], t);
          TW[c] = t;
        }
#pragma unroll
        for (int c = r; c < NX; ++c) {
          T t = Pii[r][c];
#pragma unroll
          for (int q = 0; q < NX; ++q) t = my_fma(TW[q], PiL[c][q], t);
          Ps[r][c] = t;
          Ps[c][r] = t;
        }
      }
      fin = fin && finite_state(ms, Ps);
      const int64_t o = k * L + (i - 1);
      if (ms_fast) {
#pragma unroll
        for (int r = 0; r < NX; ++r) put_global(ms_fast + o * NX + r, ms[r]);
      }
      if (Ps_fast) {
#pragma unroll
        for (int r = 0; r < NN; ++r) put_global(Ps_fast + o * NN + r, Ps[r / NX][r % NX]);
      }
      if (i == 1) {
#pragma unroll
        for (int r = 0; r < NX; ++r) {
          ms1[r] = ms[r];
#pragma unroll
          for (int c = 0; c < NX; ++c) Ps1[r][c] = Ps[r][c];
        }
        if (ms_slow) {
#pragma unroll
          for (int r = 0; r < NX; ++r) put_global(ms_slow + k * NX + r, ms[r]);
        }
        if (Ps_slow) {
#pragma unroll
          for (int r = 0; r < NN; ++r) put_global(Ps_slow + k * NN + r, Ps[r / NX][r % NX]);
        }
      }
    }
  }
  if (!fin) flag |= SRTM_INFO_NONFINITE;
  if (flag && info) atomicOr(info, flag);
}

// ============================================================================ per-window models
// Time-varying model given per window: window k's F_k, Q_k drive its fast steps x_{k,1} ..
// x_{k,l} (the step from x_{k-1,l} included) and H_k, R_k give y_k. What the time-invariant path
// computes once per call (slow-rate constants, the element matrices) is computed once per window,
// by one lane, into a per-window constants block (TvLayout: window-level constants and the
// backward factors of the fast steps; the forward quantities are recomputed where they are
// used, see TvSteps) and an element record (F, D, J). The forward scan then combines whole
// elements: the level tables of the time-invariant path do not exist here.

// Per-window constants (float64 in registers, one lane, one pass over the window's fast steps):
// the block `blk` (TvLayout `lay`) and the element matrices `el` = F, D, J of the model
// (Fm, Qm, Hm, Rm). With s_i = x_{k,1} + ... + x_{k,i} and the noise covariances (x_{k,0} = 0)
// P_xx = Q_ii, P_xs = Cov(x_{k,i}, s_i), P_ss = Cov(s_i), one fast step x <- A x + w gives
//   P_xx' = A P_xx A^T + Q,  P_xs' = A P_xs + P_xx',  P_ss' = P_ss + A P_xs + (A P_xs)^T + P_xx',
// and after l steps Q_ll = P_xx, c_l = (1/l) P_xs C^T, R_x = (1/l^2) C P_ss C^T + R (eq. h-k-l-2 and
// eq. y-k-l-2: the noise parts of Cov(x_{k,l}, y_k) and Cov(y_k)); C_bar = (C/l)(Sig_l - I),
// K = c_l R_x^{-1}, F = A^l - K C_bar, D = Q_ll - K c_l^T, J = C_bar^T R_x^{-1} C_bar. At step j the
// pass also stores A^j and C Sig_j for even j, the backward factors of fast step i = l - j.
// `blk` and `el` are the window's columns (tv_column): scalar j at blk[j * cs] and el[j * cs].
template <typename T, int NX, int NY>
SRTM_DEV int tv_window_constants(const T* __restrict__ Fm, const T* __restrict__ Qm, const T* __restrict__ Hm,
                                 const T* __restrict__ Rm, int L, const TvLayout& lay, T* __restrict__ blk,
                                 T* __restrict__ el, int64_t cs) {
  int flag = 0;
  auto W = [&](int j, double v) { put_global(blk + (int64_t)j * cs, (T)v); };
  auto WE = [&](int j, double v) { put_global(el + (int64_t)j * cs, (T)v); };
  double A[NX][NX], Q[NX][NX], C[NY][NX], R[NY][NY];
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      A[r][c] = (double)gld(Fm + r * NX + c);
      Q[r][c] = (double)gld(Qm + (c >= r ? r * NX + c : c * NX + r));  // the upper triangle
    }
#pragma unroll
  for (int r = 0; r < NY; ++r) {
#pragma unroll
    for (int c = 0; c < NX; ++c) C[r][c] = (double)gld(Hm + r * NX + c);
#pragma unroll
    for (int c = 0; c < NY; ++c) R[r][c] = (double)gld(Rm + r * NY + c);
  }
  double Aj[NX][NX], Sig[NX][NX], Pxx[NX][NX], Pxs[NX][NX], Pss[NX][NX];
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      Aj[r][c] = Sig[r][c] = (r == c) ? 1.0 : 0.0;
      Pxx[r][c] = Pxs[r][c] = Pss[r][c] = 0.0;
    }
#pragma unroll 1
  for (int j = 0; j < L; ++j) {
    if ((j & 1) == 0) {  // backward factors A^j and C Sig_j (fast step i = l - j), slot j / 2
      const int so = lay.slot + (j >> 1) * lay.slot_stride;
#pragma unroll
      for (int r = 0; r < NX; ++r)
#pragma unroll
        for (int c = 0; c < NX; ++c) W(so + lay.o_As + r * NX + c, Aj[r][c]);
#pragma unroll
      for (int r = 0; r < NY; ++r)
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          double v = 0.0;
#pragma unroll
          for (int q = 0; q < NX; ++q) v += C[r][q] * Sig[q][c];
          W(so + lay.o_CS + r * NX + c, v);
        }
    }
    // one fast step of the noise covariances
    double t[NX][NX], AP[NX][NX];
    mm(A, Pxs, t);  // A P_xs
    mm(A, Pxx, AP);
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = r; c < NX; ++c) {
        double v = Q[r][c];
#pragma unroll
        for (int q = 0; q < NX; ++q) v += AP[r][q] * A[c][q];
        Pxx[r][c] = v;
        Pxx[c][r] = v;
      }
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = r; c < NX; ++c) {
        const double v = Pss[r][c] + t[r][c] + t[c][r] + Pxx[r][c];
        Pss[r][c] = v;
        Pss[c][r] = v;
      }
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NX; ++c) Pxs[r][c] = t[r][c] + Pxx[r][c];
    mm(A, Aj, t);  // A^{j+1}, Sig_{j+1}
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        Aj[r][c] = t[r][c];
        Sig[r][c] += t[r][c];
      }
  }
  // Aj = A^l, Sig = Sig_l, Pxx = Q_ll, Pxs = Cov(x_{k,l}, s_l), Pss = Cov(s_l)
  const double il = 1.0 / (double)L;
  double Cb[NY][NX], cL[NX][NY], Rx[NY][NY];
#pragma unroll
  for (int r = 0; r < NY; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < NX; ++q) v += C[r][q] * (Sig[q][c] - (q == c ? 1.0 : 0.0));
      Cb[r][c] = v * il;
    }
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NY; ++c) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < NX; ++q) v += Pxs[r][q] * C[c][q];
      cL[r][c] = v * il;
    }
  {
    double CP[NY][NX];
    mm(C, Pss, CP);
#pragma unroll
    for (int r = 0; r < NY; ++r)
#pragma unroll
      for (int c = 0; c < NY; ++c) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < NX; ++q) v += CP[r][q] * C[c][q];
        Rx[r][c] = v * il * il + R[r][c];
      }
  }
  symmetrize(Rx);
  double Rxi[NY][NY];
  if (!spd_inv(Rx, Rxi)) flag |= SRTM_INFO_INNOVATION_NOT_PD;
  double K[NX][NY], Heta[NX][NY], Fe[NX][NX], De[NX][NX], Je[NX][NX];
  mm(cL, Rxi, K);
  mm_tn(Cb, Rxi, Heta);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      double f = Aj[r][c], dd = Pxx[r][c];
#pragma unroll
      for (int q = 0; q < NY; ++q) {
        f -= K[r][q] * Cb[q][c];
        dd -= K[r][q] * cL[c][q];
      }
      Fe[r][c] = f;
      De[r][c] = dd;
    }
  mm(Heta, Cb, Je);
  symmetrize(De);
  symmetrize(Je);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      W(lay.AL + r * NX + c, Aj[r][c]);
      WE(r * NX + c, Fe[r][c]);
      WE(NX * NX + r * NX + c, De[r][c]);
      WE(2 * NX * NX + r * NX + c, Je[r][c]);
    }
#pragma unroll
  for (int r = 0; r < NY; ++r) {
#pragma unroll
    for (int c = 0; c < NX; ++c) W(lay.Cbar + r * NX + c, Cb[r][c]);
#pragma unroll
    for (int c = 0; c < NY; ++c) W(lay.Rx + r * NY + c, Rx[r][c]);
  }
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NY; ++c) {
      W(lay.cL + r * NY + c, cL[r][c]);
      W(lay.K + r * NY + c, K[r][c]);
      W(lay.Heta + r * NY + c, Heta[r][c]);
    }
  return flag;
}

// R x C scalars of a window's column (tv_column) from scalar `off` on.
template <typename T, int R, int C>
SRTM_DEV void col_get(T (&a)[R][C], const T* __restrict__ col, int off) {
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < C; ++c) a[r][c] = gld(col + (int64_t)(off + r * C + c) * TILE);
}

// Window k's filter element: (F, D, J) from its element record, d = K y_k, eta = C_bar^T R_x^{-1} y_k
// from its block (`blk` and `el` are window k's columns, tv_column); the identity element past
// the last window.
template <typename T, int NX, int NY>
SRTM_DEV void tv_element(const T* __restrict__ blk, const T* __restrict__ el, const TvLayout& lay,
                         const T* __restrict__ y, int64_t k, int64_t N, FElem<T, NX>& a) {
  if (k >= N) {
    elem_identity(a);
    return;
  }
  constexpr int NN = NX * NX;
  col_get(a.F, el, 0);
  col_get(a.D, el, NN);
  col_get(a.J, el, 2 * NN);
  T yk[NY], K[NX][NY], He[NX][NY];
  gloadv(yk, y + k * NY);
  col_get(K, blk, lay.K);
  col_get(He, blk, lay.Heta);
  mv(K, yk, a.d);
  mv(He, yk, a.e);
}

// Per tile: the window constants of every window, then the tile's aggregate a_first (x) ... (x)
// a_last under eq. op-filter by an in-place tree in LDS (TILE whole elements).
template <typename T, int NX, int NY>
SRTM_DEV void tv_reduce_body(const T* __restrict__ Fa, const T* __restrict__ Qa, const T* __restrict__ Ha,
                             const T* __restrict__ Ra, const T* __restrict__ y, int64_t N, int L, T* __restrict__ blks,
                             T* __restrict__ els, T* __restrict__ tagg, int32_t* info, int64_t tile) {
  constexpr int NN = NX * NX, NY2 = NY * NY, NXY = NX * NY, FA = 3 * NN + 2 * NX;
  extern __shared__ char smraw[];
  const Slots<T> S{reinterpret_cast<T*>(smraw), TILE};
  const TvLayout lay = make_tv_layout(NX, NY, L);
  const int bs = lay.total, es = tv_elem_size(NX);
  const int tid = threadIdx.x;
  const int64_t k = tile * TILE + tid;
  int flag = 0;
  if (k < N)
    flag |= tv_window_constants<T, NX, NY>(Fa + k * NN, Qa + k * NN, Ha + k * NXY, Ra + k * NY2, L, lay,
                                           tv_column(blks, k, bs), tv_column(els, k, es), TILE);
  FElem<T, NX> a;
  tv_element<T, NX, NY>(tv_column(blks, k, bs), tv_column(els, k, es), lay, y, k, N, a);
  st_felem(S, tid, a);
  __syncthreads();
#pragma unroll 1
  for (int p = 0; p < LOG_TILE; ++p) {
    const int sp = 1 << p;
    if (tid < (TILE >> (p + 1))) {  // pair j to thread j: the active threads fill the first waves
      const int dst = (tid << (p + 1)) + 2 * sp - 1;
      FElem<T, NX> lft, rgt, o;
      ld_felem(S, dst - sp, lft);
      ld_felem(S, dst, rgt);
      if (!elem_combine(lft, rgt, o)) flag |= SRTM_INFO_COMBINE_SINGULAR;
      st_felem(S, dst, o);
    }
    __syncthreads();
  }
  if (tid == TILE - 1) {
    FElem<T, NX> o;
    ld_felem(S, tid, o);
    T* dst = tagg + tile * FA;
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      put_global(dst + NN + r, o.d[r]);
      put_global(dst + 2 * NN + NX + r, o.e[r]);
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        put_global(dst + r * NX + c, o.F[r][c]);
        put_global(dst + NN + NX + r * NX + c, o.D[r][c]);
        put_global(dst + 2 * NN + 2 * NX + r * NX + c, o.J[r][c]);
      }
    }
  }
  if (flag && info) atomicOr(info, flag);
}

template <typename T, int NX>
SRTM_DEV void ld_felem_global(const T* __restrict__ src, FElem<T, NX>& a) {
  constexpr int NN = NX * NX;
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    a.d[r] = gld(src + NN + r);
    a.e[r] = gld(src + 2 * NN + NX + r);
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      a.F[r][c] = gld(src + r * NX + c);
      a.D[r][c] = gld(src + NN + NX + r * NX + c);
      a.J[r][c] = gld(src + 2 * NN + 2 * NX + r * NX + c);
    }
  }
}

// One workgroup of KS threads: Kogge-Stone scan of the tile aggregates (whole elements). Thread
// tau folds its chunk of 2^lchunk tiles; the prior is folded into thread 0, which makes it a
// state; at step q threads [2^q, 2^{q+1}) combine the state of thread tau - 2^q with their run and
// the others merge two runs (eq. op-filter). Each thread then walks its chunk from its exclusive
// state, writing every tile's incoming state.
template <typename T, int NX>
SRTM_DEV void tv_tiles_body(const T* __restrict__ tagg, int64_t nt, int lchunk, int steps, const T* __restrict__ m0,
                            const T* __restrict__ P0, T* __restrict__ tstate, int32_t* info) {
  constexpr int NN = NX * NX, ST = NX + NN, FA = 3 * NN + 2 * NX;
  extern __shared__ char smraw[];
  const Slots<T> S{reinterpret_cast<T*>(smraw), KS};
  const int tid = threadIdx.x;
  const int64_t c = int64_t(1) << lchunk;
  const int64_t t0 = tid * c;
  int flag = 0;
  FElem<T, NX> run;
  elem_identity(run);
  T m[NX], P[NX][NX];  // a state once the thread's run reaches back to the prior
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    m[r] = T(0);
#pragma unroll
    for (int cc = 0; cc < NX; ++cc) P[r][cc] = T(0);
  }
#pragma unroll 1
  for (int64_t j = 0; j < c; ++j) {
    const int64_t t = t0 + j;
    if (t >= nt) break;
    FElem<T, NX> b;
    ld_felem_global(tagg + t * FA, b);
    if (j == 0) {
      run = b;
    } else if (!elem_combine(run, b, run)) {
      flag |= SRTM_INFO_COMBINE_SINGULAR;
    }
  }
  if (tid == 0) {
    gloadv(m, m0);
    gload(P, P0);
    symmetrize(P);
    if (!state_combine(m, P, run.F, run.d, run.D, run.e, run.J)) flag |= SRTM_INFO_COMBINE_SINGULAR;
  }
#pragma unroll 1
  for (int q = 0; q < steps; ++q) {
    const int sp = 1 << q;
    if (tid < sp) {
      st_state<T, NX>(S, tid, m, P);
    } else {
      st_felem(S, tid, run);
    }
    __syncthreads();
    if (tid >= sp && tid < 2 * sp) {
      ld_state<T, NX>(S, tid - sp, m, P);
      if (!state_combine(m, P, run.F, run.d, run.D, run.e, run.J)) flag |= SRTM_INFO_COMBINE_SINGULAR;
    } else if (tid >= 2 * sp) {
      FElem<T, NX> lft;
      ld_felem(S, tid - sp, lft);
      if (!elem_combine(lft, run, run)) flag |= SRTM_INFO_COMBINE_SINGULAR;
    }
    __syncthreads();
  }
  st_state<T, NX>(S, tid, m, P);  // every thread now holds the inclusive state through its chunk
  __syncthreads();
  if (t0 < nt) {
    T X[NX], XP[NX][NX];
    if (tid == 0) {
      gloadv(X, m0);
      gload(XP, P0);
      symmetrize(XP);
    } else {
      ld_state<T, NX>(S, tid - 1, X, XP);
    }
#pragma unroll 1
    for (int64_t t = t0; t < t0 + c && t < nt; ++t) {
#pragma unroll
      for (int r = 0; r < NX; ++r) put_global(tstate + t * ST + r, X[r]);
#pragma unroll
      for (int r = 0; r < NX; ++r)
#pragma unroll
        for (int cc = 0; cc < NX; ++cc) put_global(tstate + t * ST + NX + r * NX + cc, XP[r][cc]);
      if (t + 1 < t0 + c && t + 1 < nt) {
        FElem<T, NX> b;
        ld_felem_global(tagg + t * FA, b);
        if (!state_combine(X, XP, b.F, b.d, b.D, b.e, b.J)) flag |= SRTM_INFO_COMBINE_SINGULAR;
      }
    }
  }
  if (flag && info) atomicOr(info, flag);
}

// Per tile: an in-tile inclusive Kogge-Stone scan of the windows' elements, then each window's
// exclusive and inclusive filter states from the tile's incoming state; the carry (and slow
// filter outputs); with SMOOTH the smoother half of the fused kernel, with the next window's
// F and Q as the model of the step into x_{k+1,1}.
template <typename T, int NX, int NY, bool SMOOTH>
SRTM_DEV void tv_fwd_body(const T* __restrict__ Fa, const T* __restrict__ Qa, const T* __restrict__ Ha,
                          const T* __restrict__ y, int64_t N,
                          int L, const T* __restrict__ blks, const T* __restrict__ els, const T* __restrict__ m0,
                          const T* __restrict__ P0, const T* __restrict__ ftstate, T* __restrict__ carry,
                          T* __restrict__ m_slow, T* __restrict__ P_slow, T* __restrict__ btagg, T* __restrict__ sfx,
                          int32_t* info, int64_t tile) {
  constexpr int NN = NX * NX, ST = NX + NN;
  extern __shared__ char smraw[];
  const Slots<T> S{reinterpret_cast<T*>(smraw), TILE};
  const TvLayout lay = make_tv_layout(NX, NY, L);
  const int tid = threadIdx.x;
  const int64_t k = tile * TILE + tid;
  const bool valid = k < N;
  const int64_t kc = valid ? k : 0;
  int flag = 0;
  const int bs = lay.total, es = tv_elem_size(NX);
  FElem<T, NX> a, x;
  tv_element<T, NX, NY>(tv_column(blks, k, bs), tv_column(els, k, es), lay, y, k, N, a);
  x = a;
#pragma unroll 1
  for (int sp = 1; sp < TILE; sp *= 2) {  // x <- a_first (x) ... (x) a_k
    st_felem(S, tid, x);
    __syncthreads();
    FElem<T, NX> lft;
    if (tid >= sp) ld_felem(S, tid - sp, lft);
    __syncthreads();
    if (tid >= sp && !elem_combine(lft, x, x)) flag |= SRTM_INFO_COMBINE_SINGULAR;
  }
  st_felem(S, tid, x);
  __syncthreads();
  T mprev[NX], Pprev[NX][NX], m[NX], P[NX][NX];
  {
    gloadv(mprev, ftstate + tile * ST);
    gload(Pprev, ftstate + tile * ST + NX);
    symmetrize(Pprev);
    if (tid > 0) {
      FElem<T, NX> ex;
      ld_felem(S, tid - 1, ex);
      if (!state_combine(mprev, Pprev, ex.F, ex.d, ex.D, ex.e, ex.J)) flag |= SRTM_INFO_COMBINE_SINGULAR;
    }
    if (k == 0) {  // the prior itself
      gloadv(mprev, m0);
      gload(Pprev, P0);
      symmetrize(Pprev);
    }
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      m[r] = mprev[r];
#pragma unroll
      for (int c = 0; c < NX; ++c) P[r][c] = Pprev[r][c];
    }
    if (!state_combine(m, P, a.F, a.d, a.D, a.e, a.J)) flag |= SRTM_INFO_COMBINE_SINGULAR;
  }
  if (valid) flag |= store_carry(k, m, P, carry, m_slow, P_slow);
  if constexpr (SMOOTH) {
    __syncthreads();  // the slots switch from forward elements to smoother elements
    const TvModel<T, NX, NY> M{tv_tile_base(blks, k, bs), lay, (int)(k % TILE), Fa + kc * NN, Qa + kc * NN,
                               Ha + kc * NX * NY};
    T yt[NY];
#pragma unroll
    for (int r = 0; r < NY; ++r) yt[r] = valid ? gld(y + k * NY + r) : T(0);
    T An[NX][NX], Qn[NX][NX];
    const int64_t kn = (k + 1 < N) ? k + 1 : kc;  // the last window's element ignores them
    gload(An, Fa + kn * NN);
    gload(Qn, Qa + kn * NN);
    Window<T, NX, NY> w;
    if (!window_setup(M, L, mprev, Pprev, yt, w) && valid) flag |= SRTM_INFO_INNOVATION_NOT_PD;
    flag |= smoother_part<false>(M, S, L, k, N, w, m, P, An, Qn, btagg, sfx, tile);
  }
  if (flag && info) atomicOr(info, flag);
}

// ============================================================================ lag-one cross-covariances
// U_i = A^i V + c_i, the cross-covariance of x_{k,i} with y_k given y_{1:k-1}.
template <typename T, int NX, int NY>
SRTM_DEV void window_U(const Model<T, NX, NY>& M, const Window<T, NX, NY>& w, int i, T (&Ui)[NX][NY]) {
  const T* pi = M.per_i(i);
  T Ai[NX][NX], ci[NX][NY];
  load(Ai, pi + M.lay.o_Ai);
  load(ci, pi + M.lay.o_ci);
  mm(Ai, w.V, Ui);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NY; ++c) Ui[r][c] += ci[r][c];
}

// Across the window boundary, x_{k-1,l} (x_0 for the first window) given x_{k,1}, with (m, P) the
// filter state of x_{k-1,l}: the one-step smoother gain G = P A^T (P^-)^{-1}, P^- = A P A^T + Q,
// E[x_{k-1,l} | y_{1:N}] = m + G (m^s_{k,1} - A m) and Cov(x_{k,1}, x_{k-1,l} | y_{1:N}) = P^s_{k,1} G^T
// (eq. seq-smoothing-all for one step). Returns false when P^- is singular.
template <typename T, int NX>
SRTM_DEV bool lag1_boundary(const T (&A)[NX][NX], const T (&Qq)[NX][NX], const T (&m)[NX], const T (&P)[NX][NX],
                            const T (&ms)[NX], const T (&Ps)[NX][NX], T (&G)[NX][NX], T (&Pm)[NX][NX], T (&mb)[NX],
                            T (&C)[NX][NX]) {
  T Pmi[NX][NX], PA[NX][NX];
  sandwich(A, P, Qq, Pm);
  const bool ok = spd_inv(Pm, Pmi);
  mm_nt(P, A, PA);
  mm(PA, Pmi, G);
  T Am[NX], dm[NX];
  mv(A, m, Am);
#pragma unroll
  for (int r = 0; r < NX; ++r) dm[r] = ms[r] - Am[r];
  mv(G, dm, mb);
#pragma unroll
  for (int r = 0; r < NX; ++r) mb[r] += m[r];
  mm_nt(Ps, G, C);
  return ok;
}

// Inside window k, fast step i >= 2: Cov(x_{k,i}, x_{k,i-1} | y_{1:k}) = A P^f_{i-1,i-1}
// + (A c_{i-1} - c_i) S^{-1} U_{i-1}^T (x_{k,i} = A x_{k,i-1} + w, conditioned on y_k), plus the smoothing
// term P^f_{i,l} W P^f_{i-1,l}^T (PLW = P^f_{i,l} W): Cov(x_{k,i}, x_{k,i-1} | y_{1:N}).
template <typename T, int NX, int NY>
SRTM_DEV void lag1_within(const Model<T, NX, NY>& M, const Window<T, NX, NY>& w, int i, const T (&A)[NX][NX],
                          const T (&Pprev)[NX][NX], const T (&Uprev)[NX][NY], const T (&PLW)[NX][NX],
                          const T (&PLprev)[NX][NX], T (&C)[NX][NX]) {
  T Dc[NX][NY], SU[NY][NX];
  {
    T cp[NX][NY], ci[NX][NY];
    load(cp, M.per_i(i - 1) + M.lay.o_ci);
    load(ci, M.per_i(i) + M.lay.o_ci);
    mm(A, cp, Dc);
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NY; ++c) Dc[r][c] -= ci[r][c];
  }
#pragma unroll
  for (int r = 0; r < NY; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      T t = T(0);
#pragma unroll
      for (int q = 0; q < NY; ++q) t = my_fma(symget(w.Si, r, q), Uprev[c][q], t);
      SU[r][c] = t;
    }
  mm(A, Pprev, C);
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) {
      T t = C[r][c];
#pragma unroll
      for (int q = 0; q < NY; ++q) t = my_fma(Dc[r][q], SU[q][c], t);
#pragma unroll
      for (int q = 0; q < NX; ++q) t = my_fma(PLW[r][q], PLprev[c][q], t);
      C[r][c] = t;
    }
}

// K8 (optional output): per tile, the lag-one smoothed cross-covariances of every fast step of
// its windows, Cs_fast[k][i-1] = Cov(x_{k,i}, x_{k,i-1} | y_{1:N}) with x_{k,0} = x_{k-1,l} and the prior
// state x_0 for the first window (Remark cross-covariances), from the same window quantities,
// carry and smoother correction (v, W) as the recovery; records staged and written as K7's.
template <typename T, int NX, int NY>
SRTM_DEV void lag1_body(const T* __restrict__ y, int64_t N, int L, const T* __restrict__ cst,
                        const T* __restrict__ m0, const T* __restrict__ P0, const T* __restrict__ carry,
                        const T* __restrict__ sfx, const T* __restrict__ tin, T* __restrict__ Cs_fast,
                        int32_t* info, int64_t tile) {
  constexpr int NN = NX * NX, ST = NX + NN, SF = sfx_stride(NX);
  static_assert(TILE == 256, "one workgroup per tile");
  using Stg = OutStage<T, NX>;
  extern __shared__ char smraw[];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t k = tile * TILE + tid;
  const int64_t w0 = tile * TILE + wv * 64;
  const Model<T, NX, NY> M{cst, make_const_layout(NX, NY, L)};
  const int nvalid = (int)((N - w0) < 64 ? ((N - w0) > 0 ? (N - w0) : 0) : 64);
  const Stg stg(smraw + (size_t)wv * Stg::BYTES);
  const bool valid = k < N;
  const int64_t kc = valid ? k : 0;
  T m[NX], P[NX][NX], yk[NY];
  load_prior<T, NX, NY>(carry, m0, P0, kc, m, P);
  gloadv(yk, y + kc * NY);
  Window<T, NX, NY> w;
  int flag = 0;
  if (!window_setup(M, L, m, P, yk, w) && valid) flag |= SRTM_INFO_INNOVATION_NOT_PD;
  T v[NX], W[NX][NX];  // v = Et m_in + gt,  W = Et P_in Et^T + St
  {
    const T* src = sfx + kc * SF;
    const T* ti = tin + tile * ST;
    T Et[NX][NX], mi[NX], Pi[NX][NX], EP[NX][NX];
    gload(Et, src);
    gloadv(mi, ti);
    gload(Pi, ti + NX);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      T t = gld(src + NN + r);
#pragma unroll
      for (int q = 0; q < NX; ++q) t = my_fma(Et[r][q], mi[q], t);
      v[r] = t;
    }
    mm(Et, Pi, EP);
    int o = NN + NX;
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = r; c < NX; ++c) {
        T t = gld(src + o++);
#pragma unroll
        for (int q = 0; q < NX; ++q) t = my_fma(EP[r][q], Et[c][q], t);
        W[r][c] = t;
        W[c][r] = t;
      }
  }
  T A[NX][NX];
  load(A, M.cst + M.lay.A);
  T Pprev[NX][NX], PLprev[NX][NX], Uprev[NX][NY];
  const T zero[NX] = {};
  bool fin = true;
#pragma unroll 1
  for (int i = 1; i <= L; ++i) {
    T mf[NX], Pii[NX][NX], PiL[NX][NX], PLW[NX][NX], C[NX][NX];
    window_step<T, NX, NY, true>(M, w, i, mf, Pii, PiL);
    mm(PiL, W, PLW);
    if (i == 1) {  // across the window boundary, from the smoothed block of x_{k,1}
      T ms[NX], Ps[NX][NX], Qq[NX][NX], G[NX][NX], Pm[NX][NX], mb[NX];
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        T t = mf[r];
#pragma unroll
        for (int q = 0; q < NX; ++q) t = my_fma(PiL[r][q], v[q], t);
        ms[r] = t;
#pragma unroll
        for (int c = r; c < NX; ++c) {
          T u = Pii[r][c];
#pragma unroll
          for (int q = 0; q < NX; ++q) u = my_fma(PLW[r][q], PiL[c][q], u);
          Ps[r][c] = u;
          Ps[c][r] = u;
        }
      }
      load(Qq, M.cst + M.lay.Q);
      if (!lag1_boundary(A, Qq, m, P, ms, Ps, G, Pm, mb, C) && valid) flag |= SRTM_INFO_PRED_SINGULAR;
    } else {
      lag1_within(M, w, i, A, Pprev, Uprev, PLW, PLprev, C);
    }
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NX; ++c) fin = fin && isfinite(C[r][c]);
    window_U(M, w, i, Uprev);
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        Pprev[r][c] = Pii[r][c];
        PLprev[r][c] = PiL[r][c];
      }
    stg.put(lane, i, zero, C);
    wave_sync();
    stg.flush(lane, nvalid, nullptr, Cs_fast, w0, L, i, L);
    wave_sync();
  }
  if (!fin && valid) flag |= SRTM_INFO_NONFINITE;
  if (flag && info) atomicOr(info, flag);
}

// ============================================================================ log-likelihood and gradient
// Marginal log-likelihood log p(y_{1:N}) = sum_k log N(y_k; C_bar m^f_{k-1,l}, S_k) (the IMKF
// prediction of y_k, eq. m-h-k-l), and its gradient with respect to F, Q and R by Fisher's
// identity: the gradient of log p(y | theta) is the expectation, under the smoothing
// distribution, of the gradient of the complete-data log-density
//   log p(x_0) + sum_t log N(x_t; F x_{t-1}, Q) + sum_k log N(y_k; (H/l) sum_i x_{k,i}, R).
// Written with the process noise w_t = x_t - F x_{t-1} and the measurement residual
// r_k = y_k - H xbar_k (xbar_k the window average):
//   dll/dF = Q^{-1} sum_t E[w_t x_{t-1}^T],
//   dll/dQ = 1/2 Q^{-1} sum_t (E[w_t w_t^T] - Q) Q^{-1},   dll/dR = 1/2 R^{-1} sum_k (E[r_k r_k^T] - R) R^{-1}
// (expectations under p(. | y_{1:N}); symmetric-matrix gradients for Q and R: dll = tr(G dQ)).
// The summands are formed per fast step directly in their centred form, from quantities that
// scale with Q and R, never as differences of second moments of the states: near the data's
// own parameters the sums nearly vanish, and differences of state moments would carry the
// rounding of the states into the gradient multiplied by the number of steps.
//
// Per window k, with the window prior (m, P) of x_{k,0} = x_{k-1,l}, S, e and U_i as in
// eq. update-fast, the noise w_i = x_{k,i} - F x_{k,i-1} of fast step i has
//   Cov(w_i, y_k | y_{1:k-1}) = b_i = c_i - F c_{i-1}   (c_0 = 0),
//   Cov(w_i, x_{k,l} | y_{1:k}) = K_i = Q (F^{l-i})^T - b_i S^{-1} U_l^T,
// and the future measurements reach the window only through x_{k,l} (the smoother correction
// v_k, W_k of eq. seq-smoothing-all), so under p(. | y_{1:N}):
//   E[w_i] = mu_i = b_i S^{-1} e + K_i v,   E[w_i w_i^T] - Q = -b_i S^{-1} b_i^T + K_i W K_i^T + mu_i mu_i^T,
//   E[w_i x_{k,i-1}^T] = -b_i S^{-1} U_{i-1}^T + K_i W P^f_{k,i-1,l}^T + mu_i m^s_{k,i-1}^T
// with U_0 = P C_bar^T, P^f_{k,0,l} = P F^{lT} - U_0 S^{-1} U_l^T and m^s_{k,i-1} = m^f_{k,i-1} + P^f_{k,i-1,l} v.
// The measurement residual: E[r_k] = R S^{-1} e - Z v and E[r_k r_k^T] - R = E[r_k] E[r_k]^T - R S^{-1} R
// + Z W Z^T with Z = R S^{-1} U_l^T.
// These statistics are computed in float64 for both element types, from the float64 copy of the
// model constants and the stored carry and smoother correction.
//
// Per-tile record (float64): ll, then (gradient) the tile sums of E[w w^T] - Q, E[w x^T] and
// E[r r^T] - R.
template <int NX, int NY>
struct StatLayout {
  static constexpr int NN = NX * NX;
  static constexpr int LL = 0, SW = 1, SWX = 1 + NN, SY = 1 + 2 * NN, SIZE = SY + NY * NY;
};

template <typename T, int N>
SRTM_DEV T det_small(const T (&a)[N][N]) {
  static_assert(N >= 1 && N <= 2, "det_small: N <= 2");
  if constexpr (N == 1)
    return a[0][0];
  else
    return a[0][0] * a[1][1] - a[0][1] * a[1][0];
}

// Wave-wide sum (fixed butterfly order, identical on every lane).
SRTM_DEV double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T, int R, int C>
SRTM_DEV void gload_f64(double (&a)[R][C], const T* __restrict__ p) {
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < C; ++c) a[r][c] = (double)gld(p + r * C + c);
}
template <typename T, int R>
SRTM_DEV void gloadv_f64(double (&a)[R], const T* __restrict__ p) {
#pragma unroll
  for (int r = 0; r < R; ++r) a[r] = (double)gld(p + r);
}

// Gradient statistics of window k (float64), added to Sw, Swx, Sy; the window's log-likelihood
// term in *ll. (m, P): its prior; yk: its measurement (y_k - mu_k with known inputs); sfx, tin: its
// smoother-correction record and its tile's incoming smoothed state (element type T); with known
// inputs Bm [nx][nu] and uk, the window's inputs [L][nu].
template <typename T, int NX, int NY>
SRTM_DEV bool grad_window(const Model<double, NX, NY>& M, int L, const double (&m)[NX], const double (&P)[NX][NX],
                          const double (&yk)[NY], const double (&R)[NY][NY], const T* __restrict__ src,
                          const T* __restrict__ ti, double& ll, double (&Sw)[NX][NX], double (&Swx)[NX][NX],
                          double (&Sy)[NY][NY], const T* __restrict__ Bm = nullptr, const T* __restrict__ uk = nullptr,
                          int nu = 0) {
  constexpr int NN = NX * NX;
  Window<double, NX, NY> w;
  const bool ok = window_setup(M, L, m, P, yk, w);
  double e[NY];
  {
    double Cb[NY][NX];
    M.get(Cb, M.lay.Cbar);
    double quad = 0.0;
#pragma unroll
    for (int r = 0; r < NY; ++r) {
      double t = yk[r];
#pragma unroll
      for (int c = 0; c < NX; ++c) t = fma(-Cb[r][c], m[c], t);
      e[r] = t;
      quad += t * w.Se[r];
    }
    ll = -0.5 * (quad - log(det_small(w.Si)) + NY * 1.8378770664093453);  // log(2 pi)
  }
  // v = Et m_in + gt, W = Et P_in Et^T + St
  double v[NX], W[NX][NX];
  {
    double Et[NX][NX], mi[NX], Pi[NX][NX], EP[NX][NX];
    gload_f64(Et, src);
    gloadv_f64(mi, ti);
    gload_f64(Pi, ti + NX);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double t = (double)gld(src + NN + r);
#pragma unroll
      for (int q = 0; q < NX; ++q) t = fma(Et[r][q], mi[q], t);
      v[r] = t;
    }
    mm(Et, Pi, EP);
    int o = NN + NX;
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = r; c < NX; ++c) {
        double t = (double)gld(src + o++);
#pragma unroll
        for (int q = 0; q < NX; ++q) t = fma(EP[r][q], Et[c][q], t);
        W[r][c] = t;
        W[c][r] = t;
      }
  }
  double A[NX][NX], Qm[NX][NX];
  M.get(A, M.lay.A);
  M.get(Qm, M.lay.Q);
  // step i-1 quantities: U_{i-1}, P^f_{k,i-1,l}, m^f_{k,i-1}, c_{i-1}; zin: input response z_{i-1}
  double Up[NX][NY], PLp[NX][NX], mfp[NX], cp[NX][NY], zin[NX];
#pragma unroll
  for (int r = 0; r < NX; ++r) {
    zin[r] = 0.0;
    mfp[r] = w.mp[r];
#pragma unroll
    for (int c = 0; c < NY; ++c) {
      Up[r][c] = w.V[r][c];
      cp[r][c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < NX; ++c) PLp[r][c] = w.Y1[r][c];
  }
#pragma unroll 1
  for (int i = 1; i <= L; ++i) {
    double ci[NX][NY], b[NX][NY], Kq[NX][NX];
    M.get(ci, M.per_i_off(i) + M.lay.o_ci);
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NY; ++c) {
        double t = ci[r][c];
#pragma unroll
        for (int q = 0; q < NX; ++q) t = fma(-A[r][q], cp[q][c], t);
        b[r][c] = t;
      }
    // K_i = Q (A^{l-i})^T - b_i Y2 (Y2 = S^{-1} U_l^T)
    if (i < L) {
      double As[NX][NX];
      M.get(As, M.per_i_off(L - i) + M.lay.o_Ai);
      mm_nt(Qm, As, Kq);
    } else {
#pragma unroll
      for (int r = 0; r < NX; ++r)
#pragma unroll
        for (int c = 0; c < NX; ++c) Kq[r][c] = Qm[r][c];
    }
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        double t = Kq[r][c];
#pragma unroll
        for (int q = 0; q < NY; ++q) t = fma(-b[r][q], w.Y2[q][c], t);
        Kq[r][c] = t;
      }
    double bS[NX][NY], mu[NX], KW[NX][NX], msp[NX];
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NY; ++c) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < NY; ++q) t = fma(b[r][q], symget(w.Si, q, c), t);
        bS[r][c] = t;
      }
    mm(Kq, W, KW);
#pragma unroll
    for (int r = 0; r < NX; ++r) {
      double t = 0.0, s2 = mfp[r];
#pragma unroll
      for (int q = 0; q < NY; ++q) t = fma(b[r][q], w.Se[q], t);
#pragma unroll
      for (int q = 0; q < NX; ++q) {
        t = fma(Kq[r][q], v[q], t);
        s2 = fma(PLp[r][q], v[q], s2);
      }
      mu[r] = t;
      msp[r] = s2;
    }
#pragma unroll
    for (int r = 0; r < NX; ++r)
#pragma unroll
      for (int c = 0; c < NX; ++c) {
        double sw = mu[r] * mu[c], sx = mu[r] * msp[c];
#pragma unroll
        for (int q = 0; q < NY; ++q) {
          sw = fma(-bS[r][q], b[c][q], sw);
          sx = fma(-bS[r][q], Up[c][q], sx);
        }
#pragma unroll
        for (int q = 0; q < NX; ++q) {
          sw = fma(KW[r][q], Kq[c][q], sw);
          sx = fma(KW[r][q], PLp[c][q], sx);
        }
        Sw[r][c] += sw;
        Swx[r][c] += sx;
      }
    // step i's own blocks for the next step; with known inputs the fast-step means also carry the
    // input response z_i = A z_{i-1} + B u_{k,i-1} (z_0 = 0), the noise statistics do not change
    if (i < L) {
      double Pii[NX][NX];
      window_step<double, NX, NY, true>(M, w, i, mfp, Pii, PLp);
      window_U(M, w, i, Up);
      if (uk) {
        double nz[NX];
#pragma unroll
        for (int r = 0; r < NX; ++r) {
          double t = 0.0;
#pragma unroll
          for (int j = 0; j < NU_MAX; ++j)
            if (j < nu) t = fma((double)gld(Bm + r * nu + j), (double)gld(uk + (i - 1) * nu + j), t);
#pragma unroll
          for (int q = 0; q < NX; ++q) t = fma(A[r][q], zin[q], t);
          nz[r] = t;
        }
#pragma unroll
        for (int r = 0; r < NX; ++r) {
          zin[r] = nz[r];
          mfp[r] += zin[r];
        }
      }
#pragma unroll
      for (int r = 0; r < NX; ++r)
#pragma unroll
        for (int c = 0; c < NY; ++c) cp[r][c] = ci[r][c];
    }
  }
  // measurement residual: E[r] = R S^{-1} e - Z v, E[r r^T] - R = E[r]E[r]^T - R S^{-1} R + Z W Z^T
  {
    double RSi[NY][NY], Z[NY][NX], d[NY], ZW[NY][NX], Si[NY][NY];
#pragma unroll
    for (int r = 0; r < NY; ++r)
#pragma unroll
      for (int c = 0; c < NY; ++c) Si[r][c] = symget(w.Si, r, c);
    mm(R, Si, RSi);
    mm(R, w.Y2, Z);
    mm(Z, W, ZW);
#pragma unroll
    for (int r = 0; r < NY; ++r) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < NY; ++q) t = fma(RSi[r][q], e[q], t);
#pragma unroll
      for (int q = 0; q < NX; ++q) t = fma(-Z[r][q], v[q], t);
      d[r] = t;
    }
#pragma unroll
    for (int r = 0; r < NY; ++r)
#pragma unroll
      for (int c = 0; c < NY; ++c) {
        double t = d[r] * d[c];
#pragma unroll
        for (int q = 0; q < NY; ++q) t = fma(-RSi[r][q], R[q][c], t);
#pragma unroll
        for (int q = 0; q < NX; ++q) t = fma(ZW[r][q], Z[c][q], t);
        Sy[r][c] += t;
      }
  }
  return ok;
}

template <typename T, int NX, int NY, bool GRAD, bool INP>
SRTM_DEV void stats_body(const T* __restrict__ y, int64_t N, int L, const T* __restrict__ cst,
                         const double* __restrict__ cst64, InputView<T> in, const T* __restrict__ Rm,
                         const T* __restrict__ m0, const T* __restrict__ P0, const T* __restrict__ carry,
                         const T* __restrict__ sfx, const T* __restrict__ tin, double* __restrict__ parts,
                         int32_t* info, int64_t tile) {
  using SL = StatLayout<NX, NY>;
  constexpr int NN = NX * NX, ST = NX + NN, SF = sfx_stride(NX), NC = SL::SIZE;
  __shared__ double red[TILE / 64][NC];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t k = tile * TILE + tid;
  const bool valid = k < N;
  const int64_t kc = valid ? k : 0;
  double* part = parts + tile * SL::SIZE;
  int flag = 0;
  double ll = 0.0;
  double Sw[NX][NX], Swx[NX][NX], Sy[NY][NY];
#pragma unroll
  for (int r = 0; r < NX; ++r)
#pragma unroll
    for (int c = 0; c < NX; ++c) Sw[r][c] = Swx[r][c] = 0.0;
#pragma unroll
  for (int r = 0; r < NY; ++r)
#pragma unroll
    for (int c = 0; c < NY; ++c) Sy[r][c] = 0.0;
  if constexpr (GRAD) {
    const Model<double, NX, NY> M{cst64, make_const_layout(NX, NY, L)};
    double m[NX], P[NX][NX], yk[NY], R[NY][NY];
    if (kc == 0) {
      gloadv_f64(m, m0);
      gload_f64(P, P0);
    } else {
      gloadv_f64(m, carry + (kc - 1) * ST);
      gload_f64(P, carry + (kc - 1) * ST + NX);
    }
    if constexpr (INP) {  // y_k - mu_k from the tile reductions' per-window record
      gloadv_f64(yk, in.rec + kc * (NY + NX));
    } else {
      gloadv_f64(yk, y + kc * NY);
    }
    gload_f64(R, Rm);
    if (!grad_window<T, NX, NY>(M, L, m, P, yk, R, sfx + kc * SF, tin + tile * ST, ll, Sw, Swx, Sy,
                                INP ? in.B : nullptr, INP ? in.u + kc * L * in.nu : nullptr, INP ? in.nu : 0) &&
        valid)
      flag |= SRTM_INFO_INNOVATION_NOT_PD;
  } else {
    const Model<T, NX, NY> M{cst, make_const_layout(NX, NY, L), in};
    T m[NX], P[NX][NX], yk[NY];
    load_prior<T, NX, NY>(carry, m0, P0, kc, m, P);
    if constexpr (INP) {
      T zL[NX];
      window_meas<true>(M, y, kc, N, yk, zL);
    } else {
      gloadv(yk, y + kc * NY);
    }
    Window<T, NX, NY> w;
    if (!window_setup(M, L, m, P, yk, w) && valid) flag |= SRTM_INFO_INNOVATION_NOT_PD;
    T Cb[NY][NX];
    load(Cb, M.cst + M.lay.Cbar);
    double quad = 0.0;
#pragma unroll
    for (int r = 0; r < NY; ++r) {
      T t = yk[r];
#pragma unroll
      for (int c = 0; c < NX; ++c) t = my_fma(-Cb[r][c], m[c], t);
      quad += (double)t * (double)w.Se[r];
    }
    ll = -0.5 * (quad - log((double)det_small(w.Si)) + NY * 1.8378770664093453);  // log(2 pi)
  }
  // tile sums (fixed order: butterfly per wave, then waves 0..3)
  auto comp = [&](int c) -> double {
    if (!valid) return 0.0;
    if (c == SL::LL) return ll;
    if (c < SL::SWX) return Sw[(c - SL::SW) / NX][(c - SL::SW) % NX];
    if (c < SL::SY) return Swx[(c - SL::SWX) / NX][(c - SL::SWX) % NX];
    return Sy[(c - SL::SY) / NY][(c - SL::SY) % NY];
  };
  const int ncomp = GRAD ? NC : 1;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c >= ncomp) break;
    const double s = wave_sum(comp(c));
    if (lane == 0) red[wv][c] = s;
  }
  __syncthreads();
  for (int c = tid; c < ncomp; c += blockDim.x) {
    double s = red[0][c];
    for (int q = 1; q < TILE / 64; ++q) s += red[q][c];
    part[c] = s;
  }
  if (flag && info) atomicOr(info, flag);
}

// One workgroup per sequence: sums the tile records in a fixed order and forms the outputs
// dF = Q^{-1} Swx, dQ = 1/2 Q^{-1} Sw Q^{-1}, dR = 1/2 R^{-1} Sy R^{-1}.
template <typename T, int NX, int NY, bool GRAD>
SRTM_DEV void stats_final_body(int64_t nt, const T* __restrict__ Qm, const T* __restrict__ Rm,
                               const double* __restrict__ parts, T* __restrict__ ll_out, T* __restrict__ dF,
                               T* __restrict__ dQ, T* __restrict__ dR, int32_t* info) {
  using SL = StatLayout<NX, NY>;
  constexpr int NR = SL::SIZE, G = 16;
  __shared__ double red[256][G];
  __shared__ double tot[NR];
  const int tid = threadIdx.x;
  const int ncomp = GRAD ? NR : 1;
  for (int c0 = 0; c0 < ncomp; c0 += G) {
    double acc[G];
#pragma unroll
    for (int j = 0; j < G; ++j) acc[j] = 0.0;
    for (int64_t t = tid; t < nt; t += 256) {  // lane tid: tiles tid, tid + 256, ... in order
      const double* p = parts + t * SL::SIZE + c0;
#pragma unroll
      for (int j = 0; j < G; ++j)
        if (c0 + j < ncomp) acc[j] += p[j];
    }
#pragma unroll
    for (int j = 0; j < G; ++j) red[tid][j] = acc[j];
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
      if (tid < s) {
#pragma unroll
        for (int j = 0; j < G; ++j) red[tid][j] += red[tid + s][j];
      }
      __syncthreads();
    }
    if (tid < G && c0 + tid < ncomp) tot[c0 + tid] = red[0][tid];
    __syncthreads();
  }
  if (tid != 0) return;
  if (ll_out) ll_out[0] = (T)tot[SL::LL];
  if constexpr (GRAD) {
    double Q[NX][NX], R[NY][NY], Qi[NX][NX], Ri[NY][NY], Sw[NX][NX], Swx[NX][NX], Sy[NY][NY];
    for (int r = 0; r < NX; ++r)
      for (int c = 0; c < NX; ++c) {
        Q[r][c] = (double)Qm[r * NX + c];
        Sw[r][c] = tot[SL::SW + r * NX + c];
        Swx[r][c] = tot[SL::SWX + r * NX + c];
      }
    for (int r = 0; r < NY; ++r)
      for (int c = 0; c < NY; ++c) {
        R[r][c] = (double)Rm[r * NY + c];
        Sy[r][c] = tot[SL::SY + r * NY + c];
      }
    symmetrize(Q);
    symmetrize(R);
    symmetrize(Sw);
    symmetrize(Sy);
    int flag = 0;
    if (!spd_inv(Q, Qi)) flag |= SRTM_INFO_PRED_SINGULAR;
    if (!spd_inv(R, Ri)) flag |= SRTM_INFO_INNOVATION_NOT_PD;
    double tmp[NX][NX], G2[NX][NX];
    mm(Qi, Swx, tmp);
    for (int r = 0; r < NX; ++r)
      for (int c = 0; c < NX; ++c) dF[r * NX + c] = (T)tmp[r][c];
    mm(Qi, Sw, tmp);
    mm(tmp, Qi, G2);
    symmetrize(G2);
    for (int r = 0; r < NX; ++r)
      for (int c = 0; c < NX; ++c) dQ[r * NX + c] = (T)(0.5 * G2[r][c]);
    double RS[NY][NY], GR[NY][NY];
    mm(Ri, Sy, RS);
    mm(RS, Ri, GR);
    symmetrize(GR);
    for (int r = 0; r < NY; ++r)
      for (int c = 0; c < NY; ++c) dR[r * NY + c] = (T)(0.5 * GR[r][c]);
    if (flag && info) atomicOr(info, flag);
  }
}

// ============================================================================ kernels
// Every kernel takes the call's Batch. Kernels over sequences run one workgroup per sequence;
// kernels over tiles run one workgroup per tile of any sequence.
template <typename T, int NX, int NY>
struct Seq {  // one sequence's typed arrays and scan plan
  const T *F, *Q, *H, *R, *m0, *P0, *y;
  T *ms_fast, *Ps_fast, *ms_slow, *Ps_slow, *mf_fast, *Pf_fast, *mf_slow, *Pf_slow, *Cs_fast;
  T *cst, *ftagg, *ftst, *utree, *carry, *btagg, *btst, *sfx, *tvblk, *tvel;
  double *cst64, *hand, *stats;
  int64_t N, tile0;
  int L;
  ScanPlan plan;
  int32_t* info;
  InputView<T> in;
};

template <typename T, int NX, int NY>
SRTM_DEV Seq<T, NX, NY> seq_view(const Batch& b, int s) {
  const SeqDesc d = b.table ? b.table[s] : b.one;
  Seq<T, NX, NY> q;
  q.F = as_global<T>(d.F);
  q.Q = as_global<T>(d.Q);
  q.H = as_global<T>(d.H);
  q.R = as_global<T>(d.R);
  q.m0 = as_global<T>(d.m0);
  q.P0 = as_global<T>(d.P0);
  q.y = as_global<T>(d.y);
  q.ms_fast = as_global<T>(d.ms_fast);
  q.Ps_fast = as_global<T>(d.Ps_fast);
  q.ms_slow = as_global<T>(d.ms_slow);
  q.Ps_slow = as_global<T>(d.Ps_slow);
  q.mf_fast = as_global<T>(d.mf_fast);
  q.Pf_fast = as_global<T>(d.Pf_fast);
  q.mf_slow = as_global<T>(d.mf_slow);
  q.Pf_slow = as_global<T>(d.Pf_slow);
  q.Cs_fast = as_global<T>(d.Cs_fast);
  q.N = d.N;
  q.tile0 = d.tile0;
  q.L = d.L;
  q.plan = make_scan_plan(d.N);
  const WorkLayout wl = make_work_layout(NX, NY, d.L, d.N, sizeof(T), d.smoother != 0, d.B != nullptr, d.tv != 0);
  char* base = as_global(b.ws) + d.ws_off;
  q.cst = reinterpret_cast<T*>(base + wl.consts);
  q.cst64 = reinterpret_cast<double*>(base + wl.consts64);
  q.hand = reinterpret_cast<double*>(base + wl.chain);
  q.ftagg = reinterpret_cast<T*>(base + wl.ftile_agg);
  q.ftst = reinterpret_cast<T*>(base + wl.ftile_state);
  q.utree = reinterpret_cast<T*>(base + wl.utree);
  q.carry = reinterpret_cast<T*>(base + wl.carry);
  q.btagg = reinterpret_cast<T*>(base + wl.btile_agg);
  q.btst = reinterpret_cast<T*>(base + wl.btile_state);
  q.sfx = reinterpret_cast<T*>(base + wl.sfx);
  q.tvblk = reinterpret_cast<T*>(base + wl.tvblk);
  q.tvel = reinterpret_cast<T*>(base + wl.tvel);
  q.stats = reinterpret_cast<double*>(base + wl.stats);
  q.info = b.info ? b.info + s : nullptr;
  q.in = InputView<T>{as_global<T>(d.B), as_global<T>(d.u), q.H,
                      d.B ? reinterpret_cast<T*>(base + wl.inp) : nullptr, d.nu};
  return q;
}

SRTM_DEV int tile_sequence(const Batch& b, int64_t bid) { return b.tile_seq ? b.tile_seq[bid] : 0; }
SRTM_DEV int tile_sequence(const Batch& b) { return tile_sequence(b, blockIdx.x); }

// Stage bodies of the smoothing launches, for workgroup `bid` of the launch; the kernels below
// wrap them for one (nx, ny) pair, the mixed-pair kernels dispatch to them per workgroup.
template <typename T, int NX, int NY>
SRTM_DEV void kb_constants(const Batch& b, int64_t bid) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, (int)bid);
  constants_body<T, NX, NY>(q.F, q.Q, q.H, q.R, q.L, q.plan.nlev, q.cst, q.cst64, q.hand, q.info);
}

// Workgroups 0 .. nseq-1 continue the level chains of the sequences; the others reduce tile
// bid - nseq of the call.
template <typename T, int NX, int NY, bool INP>
SRTM_DEV void kb_fwd_reduce(const Batch& b, int64_t bid, int nseq) {
  if (bid < nseq) {
    const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, (int)bid);
    chain_tail_body<T, NX, NY>(q.cst, q.hand, q.L, q.plan.nlev, q.info);
    return;
  }
  const int64_t t = bid - nseq;
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, tile_sequence(b, t));
  fwd_reduce_body<INP, T, NX, NY>(q.y, q.N, q.cst, q.L, q.in, q.ftagg, q.utree, t - q.tile0);
}

template <typename T, int NX, int NY>
SRTM_DEV void kb_fwd_tiles(const Batch& b, int64_t bid) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, (int)bid);
  fwd_tiles_body<T, NX, NY>(q.ftagg, q.plan.nt, q.plan.lchunk, q.plan.steps, q.plan.nlev, q.cst, q.L, q.m0, q.P0,
                            q.ftst, q.info);
}

template <typename T, int NX, int NY, bool INP>
SRTM_DEV void kb_fwd_bwd(const Batch& b, int64_t bid) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, tile_sequence(b, bid));
  fwd_bwd_body<INP, T, NX, NY>(q.y, q.N, q.L, q.cst, q.in, q.m0, q.P0, q.ftst, q.utree, q.carry, q.mf_slow, q.Pf_slow,
                               q.btagg, q.sfx, q.info, bid - q.tile0);
}

template <typename T, int NX, int NY>
SRTM_DEV void kb_bwd_tiles(const Batch& b, int64_t bid) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, (int)bid);
  bwd_tiles_body<T, NX, NY>(q.btagg, q.plan.nt, q.plan.lchunk, q.plan.steps, q.btst);
}

template <typename T, int NX, int NY>
SRTM_DEV void kb_tv_reduce(const Batch& b, int64_t bid) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, tile_sequence(b, bid));
  tv_reduce_body<T, NX, NY>(q.F, q.Q, q.H, q.R, q.y, q.N, q.L, q.tvblk, q.tvel, q.ftagg, q.info, bid - q.tile0);
}

template <typename T, int NX, int NY>
SRTM_DEV void kb_tv_tiles(const Batch& b, int64_t bid) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, (int)bid);
  tv_tiles_body<T, NX>(q.ftagg, q.plan.nt, q.plan.lchunk, q.plan.steps, q.m0, q.P0, q.ftst, q.info);
}

template <typename T, int NX, int NY, bool SMOOTH>
SRTM_DEV void kb_tv_fwd(const Batch& b, int64_t bid) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, tile_sequence(b, bid));
  tv_fwd_body<T, NX, NY, SMOOTH>(q.F, q.Q, q.H, q.y, q.N, q.L, q.tvblk, q.tvel, q.m0, q.P0, q.ftst, q.carry,
                                 q.mf_slow, q.Pf_slow, q.btagg, q.sfx, q.info, bid - q.tile0);
}

// MODE 1: filter outputs only; 2: smoother outputs; 3: both. Fast-rate outputs take all L
// steps; with only the slow smoothed state requested, step 1 suffices.
template <typename T, int NX, int NY, int MODE, bool INP, bool TV = false>
SRTM_DEV void kb_recover(const Batch& b, int64_t bid) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, tile_sequence(b, bid));
  const bool fast = (MODE & 1) || q.ms_fast || q.Ps_fast;
  if (!fast && !q.ms_slow && !q.Ps_slow) return;
  recover_body<T, NX, NY, MODE, INP, TV>(q.y, q.N, q.L, fast ? q.L : 1, TV ? q.tvblk : q.cst, q.in, q.F, q.Q, q.m0,
                                         q.P0, q.carry, q.sfx, q.btst, q.mf_fast, q.Pf_fast, q.ms_fast, q.Ps_fast,
                                         q.ms_slow, q.Ps_slow, q.info, bid - q.tile0);
}

template <typename T, int NX, int NY>
__global__ void __launch_bounds__(256) k_constants(Batch b) {
  kb_constants<T, NX, NY>(b, blockIdx.x);
}

template <typename T, int NX, int NY, bool INP>
__global__ void __launch_bounds__(TILE) k_fwd_reduce(Batch b, int nseq) {
  kb_fwd_reduce<T, NX, NY, INP>(b, blockIdx.x, nseq);
}

template <typename T, int NX, int NY>
__global__ void __launch_bounds__(KS) k_fwd_tiles(Batch b) {
  kb_fwd_tiles<T, NX, NY>(b, blockIdx.x);
}

template <typename T, int NX, int NY, bool INP>
__global__ void __launch_bounds__(TILE) k_fwd_final(Batch b) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, tile_sequence(b));
  fwd_final_body<INP, T, NX, NY>(q.y, q.N, q.L, q.cst, q.in, q.m0, q.P0, q.ftst, q.utree, q.carry, q.mf_slow, q.Pf_slow, q.info,
                            (int64_t)blockIdx.x - q.tile0);
}

template <typename T, int NX, int NY, bool INP>
__global__ void __launch_bounds__(TILE) k_fwd_bwd(Batch b) {
  kb_fwd_bwd<T, NX, NY, INP>(b, blockIdx.x);
}

template <typename T, int NX, int NY>
__global__ void __launch_bounds__(KS) k_bwd_tiles(Batch b) {
  kb_bwd_tiles<T, NX, NY>(b, blockIdx.x);
}

// Per-window (time-varying) models: per-window constants and tile aggregates; the tile-level
// scan of whole elements; the fused per-tile forward (and smoother) pass.
template <typename T, int NX, int NY>
__global__ void __launch_bounds__(TILE) k_tv_reduce(Batch b) {
  kb_tv_reduce<T, NX, NY>(b, blockIdx.x);
}

template <typename T, int NX, int NY>
__global__ void __launch_bounds__(KS) k_tv_tiles(Batch b) {
  kb_tv_tiles<T, NX, NY>(b, blockIdx.x);
}

template <typename T, int NX, int NY, bool SMOOTH>
__global__ void __launch_bounds__(TILE) k_tv_fwd(Batch b) {
  kb_tv_fwd<T, NX, NY, SMOOTH>(b, blockIdx.x);
}

template <typename T, int NX, int NY, int MODE, bool INP, bool TV = false>
__global__ void __launch_bounds__(TILE) k_recover(Batch b) {
  kb_recover<T, NX, NY, MODE, INP, TV>(b, blockIdx.x);
}

// The constants block without the scan levels (the sequential comparator needs no scan), and the
// sequential comparator itself: one lane per sequence.
template <typename T, int NX, int NY>
__global__ void __launch_bounds__(256) k_constants_seq(Batch b) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, blockIdx.x);
  constants_body<T, NX, NY>(q.F, q.Q, q.H, q.R, q.L, 0, q.cst, q.cst64, q.hand, q.info);
}

template <typename T, int NX, int NY>
__global__ void __launch_bounds__(64) k_seq(Batch b, int nseq) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= nseq) return;
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, s);
  seq_body<T, NX, NY>(q.y, q.N, q.L, q.cst, q.m0, q.P0, q.carry, q.ms_fast, q.Ps_fast, q.ms_slow, q.Ps_slow, q.info);
}

template <typename T, int NX, int NY>
__global__ void __launch_bounds__(TILE) k_lag1(Batch b) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, tile_sequence(b));
  if (!q.Cs_fast) return;
  lag1_body<T, NX, NY>(q.y, q.N, q.L, q.cst, q.m0, q.P0, q.carry, q.sfx, q.btst, q.Cs_fast, q.info,
                       (int64_t)blockIdx.x - q.tile0);
}

template <typename T, int NX, int NY, bool GRAD, bool INP>
__global__ void __launch_bounds__(TILE) k_stats(Batch b) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, tile_sequence(b));
  stats_body<T, NX, NY, GRAD, INP>(q.y, q.N, q.L, q.cst, q.cst64, q.in, q.R, q.m0, q.P0, q.carry, q.sfx, q.btst,
                                   q.stats, q.info, (int64_t)blockIdx.x - q.tile0);
}

// Outputs: the given arrays (one sequence), or else, per sequence of a batch, its four output
// slots (ms_fast, Ps_fast, ms_slow, Ps_slow) hold ll, dF, dQ and dR.
template <typename T, int NX, int NY, bool GRAD>
__global__ void __launch_bounds__(256) k_stats_final(Batch b, T* ll, T* dF, T* dQ, T* dR) {
  const Seq<T, NX, NY> q = seq_view<T, NX, NY>(b, blockIdx.x);
  const bool own = ll == nullptr;
  stats_final_body<T, NX, NY, GRAD>(q.plan.nt, q.Q, q.R, q.stats, own ? q.ms_fast : ll,
                                    own ? q.Ps_fast : dF, own ? q.ms_slow : dQ, own ? q.Ps_slow : dR, q.info);
}

// ============================================================================ launchers

struct Events {
  hipEvent_t const* ev;
  int n;
  int j;
  hipError_t pre(hipStream_t s) {
    if (!ev || 2 * j + 1 >= n) return hipSuccess;
    return hipEventRecord(ev[2 * j], s);
  }
  hipError_t post(hipStream_t s) {
    hipError_t e = hipSuccess;
    if (ev && 2 * j + 1 < n) e = hipEventRecord(ev[2 * j + 1], s);
    ++j;
    return e;
  }
};

#define SRTM_CHECK_LAUNCH()                    \
  do {                                         \
    hipError_t _e = hipGetLastError();         \
    if (_e != hipSuccess) return SRTM_E_HIP;   \
  } while (0)

// One launch that is a stage of its own. In a profiled call (per-stage events given) the stage's
// two events are taken by the dispatch itself (hipExtLaunchKernelGGL), so that they time the
// kernel alone rather than also the gap before it; otherwise a plain launch (calls recorded into a
// graph carry no events).
#define SRTM_STAGE(kernel, grid, block, lds, st, ...)                                               \
  do {                                                                                             \
    if (ev.ev && 2 * ev.j + 1 < ev.n) {                                                            \
      hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)(lds), st, ev.ev[2 * ev.j],         \
                            ev.ev[2 * ev.j + 1], 0u, __VA_ARGS__);                                 \
    } else {                                                                                       \
      hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__);                               \
    }                                                                                              \
    ++ev.j;                                                                                        \
    SRTM_CHECK_LAUNCH();                                                                           \
  } while (0)

#define SRTM_EV(call)                          \
  do {                                         \
    if ((call) != hipSuccess) return SRTM_E_HIP; \
  } while (0)

constexpr size_t kMaxLdsBytes = 160 * 1024;  // LDS per workgroup on gfx950

// Dynamic LDS above 64 KiB must be allowed per kernel before launching.
inline bool allow_lds(const void* f, size_t bytes) {
  return bytes <= 65536 || hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) == hipSuccess;
}

// Grid shape of one call: `nseq` sequences, `ntiles` tiles in all, the largest window length.
struct Launch {
  unsigned nseq;
  unsigned ntiles;
  int max_L;
};

// What follows the scans: the fast-rate recovery (modes 1-3, see k_recover), the
// log-likelihood alone (REC_LL, after the forward scan) or the log-likelihood and its gradient
// (REC_GRAD, after both scans); `lo` receives the latter two.
template <typename T>
struct LikOut {
  T *ll, *dF, *dQ, *dR;
};

// INP: the call has known inputs (every sequence of it).
template <typename T, int NX, int NY, bool INP>
srtm_status launch_all(const Batch& b, const Launch& g, bool smoother, int rec_mode, hipStream_t st, Events ev,
                       LikOut<T> lo = LikOut<T>{nullptr, nullptr, nullptr, nullptr}) {
  constexpr int NN = NX * NX;
  const size_t lds0 = constants_lds_bytes(NX, NY, g.max_L);
  if (!allow_lds((const void*)k_constants<T, NX, NY>, lds0)) return SRTM_E_HIP;
  SRTM_STAGE((k_constants<T, NX, NY>), dim3(g.nseq), dim3(256), lds0, st, b);

  constexpr size_t lds_red = fwd_reduce_lds_bytes<T, NX>();
  SRTM_STAGE((k_fwd_reduce<T, NX, NY, INP>), dim3(g.ntiles + g.nseq), dim3(TILE), lds_red, st, b, (int)g.nseq);

  // slots, then the level records LOG_TILE .. nlev-1 of the longest sequence of the call
  const int nlev_max = make_scan_plan((int64_t)g.ntiles * TILE).nlev;
  const size_t lds_ft = sizeof(T) * ((size_t)KS * (NX + NN) +
                                     (size_t)(nlev_max - LOG_TILE) * make_const_layout(NX, NY, 1).lev_stride);
  if (!allow_lds((const void*)k_fwd_tiles<T, NX, NY>, lds_ft)) return SRTM_E_HIP;
  SRTM_STAGE((k_fwd_tiles<T, NX, NY>), dim3(g.nseq), dim3(KS), lds_ft, st, b);

  // output staging, then the per-step tables of up to RSTEPS fast steps
  const size_t ptab = sizeof(T) * (size_t)(g.max_L < RSTEPS ? g.max_L : RSTEPS) *
                      make_const_layout(NX, NY, g.max_L).per_i_stride;
  const size_t lds_rec = (size_t)4 * OutStage<T, NX>::BYTES * ((rec_mode == 3) ? 2 : 1) + ptab;
  if (!smoother) {
    const size_t lds_ff = sizeof(T) * (size_t)TILE * ((2 * NX > NX + NN) ? 2 * NX : NX + NN);
    if (!allow_lds((const void*)k_fwd_final<T, NX, NY, INP>, lds_ff)) return SRTM_E_HIP;
    SRTM_STAGE((k_fwd_final<T, NX, NY, INP>), dim3(g.ntiles), dim3(TILE), lds_ff, st, b);
    if (rec_mode == 1) {
      if (!allow_lds((const void*)k_recover<T, NX, NY, 1, INP>, lds_rec)) return SRTM_E_HIP;
      SRTM_STAGE((k_recover<T, NX, NY, 1, INP>), dim3(g.ntiles), dim3(TILE), lds_rec, st, b);
    } else {
      SRTM_EV(ev.pre(st));
      if (rec_mode == REC_LL) {
        hipLaunchKernelGGL((k_stats<T, NX, NY, false, INP>), dim3(g.ntiles), dim3(TILE), 0, st, b);
        SRTM_CHECK_LAUNCH();
        hipLaunchKernelGGL((k_stats_final<T, NX, NY, false>), dim3(g.nseq), dim3(256), 0, st, b, lo.ll, lo.dF,
                           lo.dQ, lo.dR);
        SRTM_CHECK_LAUNCH();
      }
      SRTM_EV(ev.post(st));
    }
    return SRTM_OK;
  }

  const size_t lds_fb = sizeof(T) * (size_t)TILE * ((2 * NN + NX > NX + NN) ? 2 * NN + NX : NX + NN);
  if (!allow_lds((const void*)k_fwd_bwd<T, NX, NY, INP>, lds_fb)) return SRTM_E_HIP;
  SRTM_STAGE((k_fwd_bwd<T, NX, NY, INP>), dim3(g.ntiles), dim3(TILE), lds_fb, st, b);

  const size_t lds_bk = sizeof(T) * (size_t)KS * (2 * NN + NX);
  if (!allow_lds((const void*)k_bwd_tiles<T, NX, NY>, lds_bk)) return SRTM_E_HIP;
  SRTM_STAGE((k_bwd_tiles<T, NX, NY>), dim3(g.nseq), dim3(KS), lds_bk, st, b);

  if (rec_mode == 2) {
    if (!allow_lds((const void*)k_recover<T, NX, NY, 2, INP>, lds_rec)) return SRTM_E_HIP;
    SRTM_STAGE((k_recover<T, NX, NY, 2, INP>), dim3(g.ntiles), dim3(TILE), lds_rec, st, b);
  } else if (rec_mode == 3 && lds_rec <= kMaxLdsBytes) {
    if (!allow_lds((const void*)k_recover<T, NX, NY, 3, INP>, lds_rec)) return SRTM_E_HIP;
    SRTM_STAGE((k_recover<T, NX, NY, 3, INP>), dim3(g.ntiles), dim3(TILE), lds_rec, st, b);
  } else {
    SRTM_EV(ev.pre(st));
    if (rec_mode == REC_GRAD) {
      hipLaunchKernelGGL((k_stats<T, NX, NY, true, INP>), dim3(g.ntiles), dim3(TILE), 0, st, b);
      SRTM_CHECK_LAUNCH();
      hipLaunchKernelGGL((k_stats_final<T, NX, NY, true>), dim3(g.nseq), dim3(256), 0, st, b, lo.ll, lo.dF, lo.dQ,
                         lo.dR);
      SRTM_CHECK_LAUNCH();
    } else if (rec_mode == 3) {  // filter and smoother staging do not fit together: two passes
      const size_t lds1 = (size_t)4 * OutStage<T, NX>::BYTES + ptab;
      if (!allow_lds((const void*)k_recover<T, NX, NY, 1, INP>, lds1)) return SRTM_E_HIP;
      if (!allow_lds((const void*)k_recover<T, NX, NY, 2, INP>, lds1)) return SRTM_E_HIP;
      hipLaunchKernelGGL((k_recover<T, NX, NY, 1, INP>), dim3(g.ntiles), dim3(TILE), lds1, st, b);
      SRTM_CHECK_LAUNCH();
      hipLaunchKernelGGL((k_recover<T, NX, NY, 2, INP>), dim3(g.ntiles), dim3(TILE), lds1, st, b);
      SRTM_CHECK_LAUNCH();
    }
    SRTM_EV(ev.post(st));
  }
  return SRTM_OK;
}

// The sequential comparator (REC_SEQ): the constants, then one lane per sequence.
template <typename T, int NX, int NY>
srtm_status launch_seq(const Batch& b, const Launch& g, hipStream_t st) {
  const size_t lds0 = constants_lds_bytes(NX, NY, g.max_L);
  if (!allow_lds((const void*)k_constants_seq<T, NX, NY>, lds0)) return SRTM_E_HIP;
  hipLaunchKernelGGL((k_constants_seq<T, NX, NY>), dim3(g.nseq), dim3(256), lds0, st, b);
  SRTM_CHECK_LAUNCH();
  hipLaunchKernelGGL((k_seq<T, NX, NY>), dim3((g.nseq + 63) / 64), dim3(64), 0, st, b, (int)g.nseq);
  SRTM_CHECK_LAUNCH();
  return SRTM_OK;
}

// Per-window (time-varying) model, one sequence: 6 launches for the smoother (k_tv_reduce,
// k_tv_tiles, k_tv_fwd<1>, k_bwd_tiles, k_recover), 4 for the filter.
template <typename T, int NX, int NY>
srtm_status launch_tv(const Batch& b, const Launch& g, bool smoother, int rec_mode, hipStream_t st) {
  if constexpr (NX > TV_NX_MAX) {
    return SRTM_E_UNSUPPORTED;
  } else {
    constexpr int NN = NX * NX, FA = 3 * NN + 2 * NX;
    const size_t lds_el = sizeof(T) * (size_t)TILE * FA;  // a tile of whole elements
    if (!allow_lds((const void*)k_tv_reduce<T, NX, NY>, lds_el)) return SRTM_E_HIP;
    hipLaunchKernelGGL((k_tv_reduce<T, NX, NY>), dim3(g.ntiles), dim3(TILE), lds_el, st, b);
    SRTM_CHECK_LAUNCH();
    const size_t lds_ks = sizeof(T) * (size_t)KS * FA;
    if (!allow_lds((const void*)k_tv_tiles<T, NX, NY>, lds_ks)) return SRTM_E_HIP;
    hipLaunchKernelGGL((k_tv_tiles<T, NX, NY>), dim3(g.nseq), dim3(KS), lds_ks, st, b);
    SRTM_CHECK_LAUNCH();
    const size_t lds_rec = (size_t)4 * OutStage<T, NX>::BYTES + tv_model_lds_bytes<T, NX, NY>();
    if (!smoother) {
      if (!allow_lds((const void*)k_tv_fwd<T, NX, NY, false>, lds_el)) return SRTM_E_HIP;
      hipLaunchKernelGGL((k_tv_fwd<T, NX, NY, false>), dim3(g.ntiles), dim3(TILE), lds_el, st, b);
      SRTM_CHECK_LAUNCH();
      if (rec_mode == 1) {
        if (!allow_lds((const void*)k_recover<T, NX, NY, 1, false, true>, lds_rec)) return SRTM_E_HIP;
        hipLaunchKernelGGL((k_recover<T, NX, NY, 1, false, true>), dim3(g.ntiles), dim3(TILE), lds_rec, st, b);
        SRTM_CHECK_LAUNCH();
      }
      return SRTM_OK;
    }
    if (!allow_lds((const void*)k_tv_fwd<T, NX, NY, true>, lds_el)) return SRTM_E_HIP;
    hipLaunchKernelGGL((k_tv_fwd<T, NX, NY, true>), dim3(g.ntiles), dim3(TILE), lds_el, st, b);
    SRTM_CHECK_LAUNCH();
    const size_t lds_bk = sizeof(T) * (size_t)KS * (2 * NN + NX);
    if (!allow_lds((const void*)k_bwd_tiles<T, NX, NY>, lds_bk)) return SRTM_E_HIP;
    hipLaunchKernelGGL((k_bwd_tiles<T, NX, NY>), dim3(g.nseq), dim3(KS), lds_bk, st, b);
    SRTM_CHECK_LAUNCH();
    if (rec_mode == 2 || rec_mode == 3) {  // filter and smoother outputs: two recovery passes
      if (rec_mode == 3) {
        if (!allow_lds((const void*)k_recover<T, NX, NY, 1, false, true>, lds_rec)) return SRTM_E_HIP;
        hipLaunchKernelGGL((k_recover<T, NX, NY, 1, false, true>), dim3(g.ntiles), dim3(TILE), lds_rec, st, b);
        SRTM_CHECK_LAUNCH();
      }
      if (!allow_lds((const void*)k_recover<T, NX, NY, 2, false, true>, lds_rec)) return SRTM_E_HIP;
      hipLaunchKernelGGL((k_recover<T, NX, NY, 2, false, true>), dim3(g.ntiles), dim3(TILE), lds_rec, st, b);
      SRTM_CHECK_LAUNCH();
    }
    return SRTM_OK;
  }
}

// One sequence (srtm_filter / srtm_smooth).
template <typename T, int NX, int NY>
srtm_status run(const srtm_shape& sh, const Ptrs& p, bool smoother, hipStream_t st, Events ev, int lik_mode = 0,
                void* ll = nullptr, void* dF = nullptr, void* dQ = nullptr, void* dR = nullptr) {
  Batch b{};
  b.table = nullptr;
  b.tile_seq = nullptr;
  b.ws = static_cast<char*>(p.ws);
  b.info = p.info;
  SeqDesc& d = b.one;
  d.F = p.F; d.Q = p.Q; d.H = p.H; d.R = p.R; d.m0 = p.m0; d.P0 = p.P0; d.y = p.y;
  d.ms_fast = p.ms_fast; d.Ps_fast = p.Ps_fast; d.ms_slow = p.ms_slow; d.Ps_slow = p.Ps_slow;
  d.mf_fast = p.mf_fast; d.Pf_fast = p.Pf_fast; d.mf_slow = p.mf_slow; d.Pf_slow = p.Pf_slow;
  d.N = sh.N;
  d.tile0 = 0;
  d.ws_off = 0;
  d.L = sh.L;
  d.smoother = smoother ? 1 : 0;
  d.B = p.B;
  d.u = p.u;
  d.nu = p.B ? p.nu : 0;
  d.tv = p.tv ? 1 : 0;
  d.Cs_fast = p.Cs_fast;
  d.nx = NX;
  d.ny = NY;
  const Launch g{1u, (unsigned)((sh.N + TILE - 1) / TILE), (int)sh.L};
  const bool want_f = p.mf_fast || p.Pf_fast;
  const bool want_s = p.ms_fast || p.Ps_fast || p.ms_slow || p.Ps_slow;
  const int mode = lik_mode ? lik_mode : (smoother ? (want_f ? 3 : (want_s ? 2 : 0)) : (want_f ? 1 : 0));
  const LikOut<T> lo{static_cast<T*>(ll), static_cast<T*>(dF), static_cast<T*>(dQ), static_cast<T*>(dR)};
  if (lik_mode == REC_SEQ) {
    if (p.tv || p.B || p.Cs_fast || ev.ev || !smoother) return SRTM_E_UNSUPPORTED;
    return launch_seq<T, NX, NY>(b, g, st);
  }
  if (p.tv) {
    if (lik_mode || ev.ev) return SRTM_E_UNSUPPORTED;  // no log-likelihood or profiling form
    return launch_tv<T, NX, NY>(b, g, smoother, mode, st);
  }
  if (p.B) return launch_all<T, NX, NY, true>(b, g, smoother, mode, st, ev, lo);
  if (!p.Cs_fast) return launch_all<T, NX, NY, false>(b, g, smoother, mode, st, ev, lo);
  // lag-one cross-covariances: the smoother's launches, then one more pass over the tiles
  if (!smoother || lik_mode || ev.ev) return SRTM_E_UNSUPPORTED;
  const srtm_status s = launch_all<T, NX, NY, false>(b, g, smoother, mode, st, ev, lo);
  if (s != SRTM_OK) return s;
  const size_t lds = (size_t)4 * OutStage<T, NX>::BYTES;
  if (!allow_lds((const void*)k_lag1<T, NX, NY>, lds)) return SRTM_E_HIP;
  hipLaunchKernelGGL((k_lag1<T, NX, NY>), dim3(g.ntiles), dim3(TILE), lds, st, b);
  SRTM_CHECK_LAUNCH();
  return SRTM_OK;
}

// Many sequences (srtm_smooth_batch): `table` holds nseq descriptors followed by the sequence
// index of every tile, in device memory.
template <typename T, int NX, int NY>
srtm_status run_batch(const void* table, int nseq, int64_t ntiles, int max_L, void* ws, int32_t* info,
                      hipStream_t st, bool grad) {
  Batch b{};
  b.table = static_cast<const SeqDesc*>(table);
  b.tile_seq = reinterpret_cast<const int32_t*>(static_cast<const char*>(table) + batch_tile_map_offset(nseq));
  b.ws = static_cast<char*>(ws);
  b.info = info;
  const Launch g{(unsigned)nseq, (unsigned)ntiles, max_L};
  return launch_all<T, NX, NY, false>(b, g, true, grad ? REC_GRAD : 2, st, Events{nullptr, 0, 0});
}

}  // namespace srtm

#if defined(SRTM_MIXED_T)
// ---------------------------------------------------------------- mixed-pair launches
// One set of six launches for a batch whose sequences differ in (nx, ny) and kind (time-invariant
// model, with known inputs, or per-window model): every workgroup reads its sequence's descriptor
// and runs that pair's and kind's stage body. Each sequence gets exactly the per-pair kernels'
// arithmetic on the same tiles. This object is compiled once per element type (SRTM_MIXED_T).
namespace srtm {

template <typename T>
__global__ void __launch_bounds__(256) km_constants(Batch b) {
  const SeqDesc& d = b.table[blockIdx.x];
  if (d.tv) return;  // per-window models build their constants per tile in the next stage
#define SRTM_MX(a, c)                          \
  if (d.nx == a && d.ny == c) {                \
    kb_constants<T, a, c>(b, blockIdx.x);      \
    return;                                    \
  }
  SRTM_PAIRS(SRTM_MX)
#undef SRTM_MX
}

// Workgroups 0 .. nseq-1: level chains (time-invariant models); the rest: tile reductions.
template <typename T>
__global__ void __launch_bounds__(TILE) km_reduce(Batch b, int nseq) {
  const int64_t bid = blockIdx.x;
  const SeqDesc& d = b.table[bid < nseq ? (int)bid : tile_sequence(b, bid - nseq)];
#define SRTM_MX(a, c)                                                    \
  if (d.nx == a && d.ny == c) {                                          \
    if (d.tv) {                                                          \
      if constexpr (a <= TV_NX_MAX) {                                    \
        if (bid >= nseq) kb_tv_reduce<T, a, c>(b, bid - nseq);           \
      }                                                                  \
    } else if (d.B) {                                                    \
      kb_fwd_reduce<T, a, c, true>(b, bid, nseq);                        \
    } else {                                                             \
      kb_fwd_reduce<T, a, c, false>(b, bid, nseq);                       \
    }                                                                    \
    return;                                                              \
  }
  SRTM_PAIRS(SRTM_MX)
#undef SRTM_MX
}

template <typename T>
__global__ void __launch_bounds__(KS) km_fwd_tiles(Batch b) {
  const SeqDesc& d = b.table[blockIdx.x];
#define SRTM_MX(a, c)                                      \
  if (d.nx == a && d.ny == c) {                            \
    if (d.tv) {                                            \
      if constexpr (a <= TV_NX_MAX) kb_tv_tiles<T, a, c>(b, blockIdx.x); \
    } else {                                               \
      kb_fwd_tiles<T, a, c>(b, blockIdx.x);                \
    }                                                      \
    return;                                                \
  }
  SRTM_PAIRS(SRTM_MX)
#undef SRTM_MX
}

template <typename T>
__global__ void __launch_bounds__(TILE) km_fwd_bwd(Batch b) {
  const SeqDesc& d = b.table[tile_sequence(b)];
#define SRTM_MX(a, c)                                                    \
  if (d.nx == a && d.ny == c) {                                          \
    if (d.tv) {                                                          \
      if constexpr (a <= TV_NX_MAX) kb_tv_fwd<T, a, c, true>(b, blockIdx.x); \
    } else if (d.B) {                                                    \
      kb_fwd_bwd<T, a, c, true>(b, blockIdx.x);                          \
    } else {                                                             \
      kb_fwd_bwd<T, a, c, false>(b, blockIdx.x);                         \
    }                                                                    \
    return;                                                              \
  }
  SRTM_PAIRS(SRTM_MX)
#undef SRTM_MX
}

template <typename T>
__global__ void __launch_bounds__(KS) km_bwd_tiles(Batch b) {
  const SeqDesc& d = b.table[blockIdx.x];
#define SRTM_MX(a, c)                          \
  if (d.nx == a && d.ny == c) {                \
    kb_bwd_tiles<T, a, c>(b, blockIdx.x);      \
    return;                                    \
  }
  SRTM_PAIRS(SRTM_MX)
#undef SRTM_MX
}

template <typename T>
__global__ void __launch_bounds__(TILE) km_recover(Batch b) {
  const SeqDesc& d = b.table[tile_sequence(b)];
#define SRTM_MX(a, c)                                                           \
  if (d.nx == a && d.ny == c) {                                                 \
    if (d.tv) {                                                                 \
      if constexpr (a <= TV_NX_MAX) kb_recover<T, a, c, 2, false, true>(b, blockIdx.x); \
    } else if (d.B) {                                                           \
      kb_recover<T, a, c, 2, true>(b, blockIdx.x);                              \
    } else {                                                                    \
      kb_recover<T, a, c, 2, false>(b, blockIdx.x);                             \
    }                                                                           \
    return;                                                                     \
  }
  SRTM_PAIRS(SRTM_MX)
#undef SRTM_MX
}

// Dynamic LDS of the six stages for one sequence of pair (NX, NY): the launch takes the largest
// over the batch's sequences.
template <typename T, int NX, int NY>
void stage_lds(bool tv, int max_L, int nlev_max, size_t (&o)[6]) {
  constexpr int NN = NX * NX;
  auto up = [&](int j, size_t v) { o[j] = v > o[j] ? v : o[j]; };
  if (!tv) {
    up(0, constants_lds_bytes(NX, NY, max_L));
    up(1, fwd_reduce_lds_bytes<T, NX>());
    up(2, sizeof(T) * ((size_t)KS * (NX + NN) + (size_t)(nlev_max - LOG_TILE) * make_const_layout(NX, NY, 1).lev_stride));
    up(3, sizeof(T) * (size_t)TILE * ((2 * NN + NX > NX + NN) ? 2 * NN + NX : NX + NN));
    up(5, (size_t)4 * OutStage<T, NX>::BYTES +
              sizeof(T) * (size_t)(max_L < RSTEPS ? max_L : RSTEPS) * make_const_layout(NX, NY, max_L).per_i_stride);
  } else {
    if constexpr (NX <= TV_NX_MAX) {
      constexpr int FA = 3 * NN + 2 * NX;
      up(1, sizeof(T) * (size_t)TILE * FA);
      up(2, sizeof(T) * (size_t)KS * FA);
      up(3, sizeof(T) * (size_t)TILE * FA);
      up(5, (size_t)4 * OutStage<T, NX>::BYTES + tv_model_lds_bytes<T, NX, NY>());
    }
  }
  up(4, sizeof(T) * (size_t)KS * (2 * NN + NX));
}

template <typename T>
srtm_status run_mixed(const SeqDesc* host, const void* table_dev, int nseq, int64_t ntiles, int max_L, void* ws,
                      int32_t* info, hipStream_t st) {
  Batch b{};
  b.table = static_cast<const SeqDesc*>(table_dev);
  b.tile_seq = reinterpret_cast<const int32_t*>(static_cast<const char*>(table_dev) + batch_tile_map_offset(nseq));
  b.ws = static_cast<char*>(ws);
  b.info = info;
  const int nlev_max = make_scan_plan(ntiles * TILE).nlev;
  size_t lds[6] = {0, 0, 0, 0, 0, 0};
  for (int s = 0; s < nseq; ++s) {
#define SRTM_MX(a, c) \
  if (host[s].nx == a && host[s].ny == c) stage_lds<T, a, c>(host[s].tv != 0, max_L, nlev_max, lds);
    SRTM_PAIRS(SRTM_MX)
#undef SRTM_MX
  }
  const void* fn[6] = {(const void*)km_constants<T>, (const void*)km_reduce<T>, (const void*)km_fwd_tiles<T>,
                       (const void*)km_fwd_bwd<T>, (const void*)km_bwd_tiles<T>, (const void*)km_recover<T>};
  for (int j = 0; j < 6; ++j)
    if (!allow_lds(fn[j], lds[j])) return SRTM_E_HIP;
  const unsigned ns = (unsigned)nseq, nt = (unsigned)ntiles;
  hipLaunchKernelGGL((km_constants<T>), dim3(ns), dim3(256), lds[0], st, b);
  SRTM_CHECK_LAUNCH();
  hipLaunchKernelGGL((km_reduce<T>), dim3(nt + ns), dim3(TILE), lds[1], st, b, nseq);
  SRTM_CHECK_LAUNCH();
  hipLaunchKernelGGL((km_fwd_tiles<T>), dim3(ns), dim3(KS), lds[2], st, b);
  SRTM_CHECK_LAUNCH();
  hipLaunchKernelGGL((km_fwd_bwd<T>), dim3(nt), dim3(TILE), lds[3], st, b);
  SRTM_CHECK_LAUNCH();
  hipLaunchKernelGGL((km_bwd_tiles<T>), dim3(ns), dim3(KS), lds[4], st, b);
  SRTM_CHECK_LAUNCH();
  hipLaunchKernelGGL((km_recover<T>), dim3(nt), dim3(TILE), lds[5], st, b);
  SRTM_CHECK_LAUNCH();
  return SRTM_OK;
}

#define SRTM_MIXED_NAME2(t) run_mixed_##t
#define SRTM_MIXED_NAME(t) SRTM_MIXED_NAME2(t)
srtm_status SRTM_MIXED_NAME(SRTM_MIXED_T)(const SeqDesc* host, const void* table_dev, int nseq, int64_t ntiles,
                                          int max_L, void* ws, int32_t* info, hipStream_t st) {
  return run_mixed<SRTM_MIXED_T>(host, table_dev, nseq, ntiles, max_L, ws, info, st);
}

}  // namespace srtm
#else
// ---------------------------------------------------------------- this object's (nx, ny) pair
#if !defined(SRTM_NX) || !defined(SRTM_NY)
#error "srtm_kernels.hip is compiled once per (nx, ny) pair (SRTM_NX, SRTM_NY) or per element type (SRTM_MIXED_T)"
#endif
#define SRTM_NAME2(p, a, b) p##a##_##b
#define SRTM_NAME(p, a, b) SRTM_NAME2(p, a, b)

namespace srtm {
srtm_status SRTM_NAME(run_pair_, SRTM_NX, SRTM_NY)(int dtype, const srtm_shape& sh, const Ptrs& p, bool smoother,
                                                   hipStream_t st, hipEvent_t const* ev, int nev, int lik_mode,
                                                   void* ll, void* dF, void* dQ, void* dR) {
  const Events E{ev, nev, 0};
  if (dtype == SRTM_F64) return run<double, SRTM_NX, SRTM_NY>(sh, p, smoother, st, E, lik_mode, ll, dF, dQ, dR);
  return run<float, SRTM_NX, SRTM_NY>(sh, p, smoother, st, E, lik_mode, ll, dF, dQ, dR);
}

srtm_status SRTM_NAME(run_batch_pair_, SRTM_NX, SRTM_NY)(int dtype, const void* table, int nseq, int64_t ntiles,
                                                         int max_L, void* ws, int32_t* info, hipStream_t st,
                                                         bool grad) {
  if (dtype == SRTM_F64) return run_batch<double, SRTM_NX, SRTM_NY>(table, nseq, ntiles, max_L, ws, info, st, grad);
  return run_batch<float, SRTM_NX, SRTM_NY>(table, nseq, ntiles, max_L, ws, info, st, grad);
}
}  // namespace srtm
#endif  // SRTM_MIXED_T
