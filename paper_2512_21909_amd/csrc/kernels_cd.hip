// Symmetry-adapted two-step Cholesky decomposition, FP64 kernels for gfx950.
//
// Paper: section "Symmetry-adapted two-step CD algorithm", Algorithm 1 (the
// Cholesky basis: diagonal screening, qualified batches of at most Q_max
// pairs with Diag >= sigma D_max, residual columns, micro iterations over
// the qualified pairs, pruning of P) and the second-step equation for the
// vectors L^P_rs = sum_R K^-1_PR (R|rs) with K K^T the metric over the basis.
// The integral matrix is given per irrep as a dense symmetric matrix V (rows
// and columns: the basis-function pairs of the irrep).
//
// First step, per macro iteration (host loop in cd.cpp):
//   gather     M[r][slot] = V[r][q_slot] for the qualified pairs q of an irrep
//   gemm_nt    M -= L1 L1[Q]^T (the vectors of earlier macro iterations)
//   argmax     pivot = the first largest Diag over Q (one workgroup)
//   column     the new vector over P: (M[r][q] - sum_mic L1[r] L1[q]) / sqrt(d)
//              and Diag(r) -= L^2; argmax and column alternate, launched in
//              chunks without host synchronisation (a device flag ends them)
// Second step, per irrep: gather the metric V[piv][piv] and Y = V[:, piv];
// blocked right-looking Cholesky of the metric (diagonal block in LDS, row
// solves of the panel, gemm_nt trailing update); then Y K^-T by 64-column
// blocks (gemm_nt update with the solved columns, row solves): L[r][P].
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"

namespace cdcc {

typedef double cd4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// first step
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cd_diag_kernel(const double *__restrict__ V, int64_t n,
                                                      double *__restrict__ D) {
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r < n) D[r] = V[r * n + r];
}

// M[r][slot] = V[r][qrows[slot]], r < n, slot < nq (ld of M = ldm).
__global__ __launch_bounds__(256) void cd_gather_cols_kernel(const double *__restrict__ V, int64_t n,
                                                             const int32_t *__restrict__ qrows, int nq,
                                                             double *__restrict__ M, int ldm) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (e >= n * nq) return;
  const int64_t r = e / nq;
  const int s = int(e - r * nq);
  M[r * ldm + s] = V[r * n + qrows[s]];
}

// One micro-iteration pivot choice over the qualified list (all irreps):
// the first maximum of Diag in Q order; below tau_mic (or Q used up) ends the
// macro iteration.
__global__ __launch_bounds__(1024) void cd_argmax_kernel(const CdQ *__restrict__ q, int nq, CdPtrs P,
                                                         CdState *__restrict__ st) {
  __shared__ double sv[1024];
  __shared__ int si[1024];
  const int tid = threadIdx.x;
  if (st->done) {
    if (tid == 0) st->step_valid = 0;
    return;
  }
  double best = -1.0 / 0.0;
  int bi = nq;
  for (int e = tid; e < nq; e += 1024) {
    const CdQ x = q[e];
    const double v = P.D[x.g][x.r];
    if (v > best) {  // e increases within a thread: the first maximum is kept
      best = v;
      bi = e;
    }
  }
  sv[tid] = best;
  si[tid] = bi;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) {
      const double v2 = sv[tid + w];
      const int i2 = si[tid + w];
      if (v2 > sv[tid] || (v2 == sv[tid] && i2 < si[tid])) {
        sv[tid] = v2;
        si[tid] = i2;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double v = sv[0];
    const int e = si[0];
    if (e >= nq || !(v >= st->tau_mic) || st->steps >= nq) {
      st->done = 1;
      st->step_valid = 0;
    } else {
      const CdQ x = q[e];
      const int col = st->k[x.g];
      st->k[x.g] = col + 1;
      P.piv[x.g][col] = x.r;
      st->cur_g = x.g;
      st->cur_r = x.r;
      st->cur_slot = x.slot;
      st->cur_col = col;
      st->cur_d = v;
      st->steps += 1;
      st->step_valid = 1;
    }
  }
}

// The new vector of the chosen pivot over the rows of its irrep.
__global__ __launch_bounds__(256) void cd_column_kernel(CdPtrs P, CdState *__restrict__ st) {
  __shared__ double lq[kCdQmaxCap];
  if (!st->step_valid) return;
  const int g = st->cur_g, col = st->cur_col, q = st->cur_r, slot = st->cur_slot;
  const int k0 = st->k0[g];
  const double d = st->cur_d;
  const int64_t n = P.n[g];
  const int nm = col - k0;
  double *__restrict__ L1 = P.L1[g];
  for (int i = threadIdx.x; i < nm; i += 256) lq[i] = L1[int64_t(q) * n + k0 + i];
  __syncthreads();
  const int64_t r = int64_t(blockIdx.x) * 256 + threadIdx.x;
  if (r >= n) return;
  if (!P.inP[g][r]) {
    L1[r * n + col] = 0.0;
    return;
  }
  double s = P.M[g][r * P.qcap[g] + slot];
  const double *__restrict__ lr = L1 + r * n + k0;
  for (int i = 0; i < nm; ++i) s -= lr[i] * lq[i];
  const double x = s / sqrt(d);
  L1[r * n + col] = x;
  P.D[g][r] = (r == q) ? 0.0 : P.D[g][r] - x * x;
}

// ---------------------------------------------------------------------------
// generic C[m][n] += alpha sum_k A[arow(m)][k] B[brow(n)][k]  (both operands
// K-contiguous rows; optional row-index tables), 64 x 64 tiles, 4 waves in
// 2 x 2 of MFMA f64 16x16x4, BK = 16 double-buffered LDS ([k][m], [k][n]).
// Rows past M / N read a clamped row and are not stored; k past K is zeroed
// by a select.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cd_gemm_nt_kernel(CdGemm G) {
  constexpr int BM = 64, BK = 16, LD = BM + 2;
  __shared__ double As[2][BK][LD], Bs[2][BK][LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BM;
  const int lr = tid >> 2, lk = (tid & 3) * 4;
  const int am = min(m0 + lr, G.M - 1), bn = min(n0 + lr, G.N - 1);
  const CDCC_GLOBAL double *arow = as_global(G.A) + int64_t(G.arows ? G.arows[am] : am) * G.lda;
  const CDCC_GLOBAL double *brow = as_global(G.B) + int64_t(G.brows ? G.brows[bn] : bn) * G.ldb;
  cd4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = cd4{0.0, 0.0, 0.0, 0.0};
  double ra[4], rb[4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + lk + e;
      const int kc = min(k, G.K - 1);
      const double x = arow[kc], y = brow[kc];
      ra[e] = k < G.K ? x : 0.0;
      rb[e] = k < G.K ? y : 0.0;
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      As[buf][lk + e][lr] = ra[e];
      Bs[buf][lk + e][lr] = rb[e];
    }
  };
  const int nkb = (G.K + BK - 1) / BK;
  if (nkb > 0) {
    gload(0);
    lstore(0);
  }
  __syncthreads();
  for (int kb = 0; kb < nkb; ++kb) {
    const int cur = kb & 1;
    const bool more = kb + 1 < nkb;
    if (more) gload((kb + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kr = ks * 4 + (lane >> 4);
      double fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        fa[i] = As[cur][kr][wm * 32 + i * 16 + (lane & 15)];
        fb[i] = Bs[cur][kr][wn * 32 + i * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
    }
    if (more) lstore(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * r;
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m < G.M && n < G.N) {
          double *c = G.C + int64_t(m) * G.ldc + n;
          *c = *c + G.alpha * acc[i][j][r];
        }
      }
}

// ---------------------------------------------------------------------------
// second step
// ---------------------------------------------------------------------------
// K[i][j] = V[piv_i][piv_j] (np x np) and Y[r][j] = V[r][piv_j] (n x np).
__global__ __launch_bounds__(256) void cd_gather_metric_kernel(const double *__restrict__ V, int64_t n,
                                                               const int32_t *__restrict__ piv, int np,
                                                               double *__restrict__ K, double *__restrict__ Y) {
  const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
  const int64_t nk = int64_t(np) * np;
  if (e < nk) {
    const int64_t i = e / np;
    const int j = int(e - i * np);
    K[e] = V[int64_t(piv[i]) * n + piv[j]];
  } else if (e < nk + n * np) {
    const int64_t f = e - nk;
    const int64_t r = f / np;
    const int j = int(f - r * np);
    Y[f] = V[r * n + piv[j]];
  }
}

// Lower Cholesky factor of the w x w block at (j0, j0) of K (ld), in place;
// a non-positive pivot sets *bad.
__global__ __launch_bounds__(256) void cd_potrf_diag_kernel(double *__restrict__ K, int ld, int j0, int w,
                                                            int *__restrict__ bad) {
  __shared__ double a[64][65];
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += 256) {
    const int i = e / w, j = e - (e / w) * w;
    a[i][j] = K[int64_t(j0 + i) * ld + j0 + j];
  }
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    const double d = a[j][j];
    __syncthreads();
    if (!(d > 0.0)) {
      if (tid == 0) *bad = 1;
      return;  // uniform: every thread read the same d
    }
    const double s = sqrt(d);
    for (int i = j + 1 + tid; i < w; i += 256) a[i][j] /= s;
    if (tid == 0) a[j][j] = s;
    __syncthreads();
    for (int e = tid; e < (w - j - 1) * (w - j - 1); e += 256) {
      const int i = j + 1 + e / (w - j - 1), k = j + 1 + e % (w - j - 1);
      if (k <= i) a[i][k] -= a[i][j] * a[k][j];
    }
    __syncthreads();
  }
  for (int e = tid; e < w * w; e += 256) {
    const int i = e / w, j = e - (e / w) * w;
    if (j <= i) K[int64_t(j0 + i) * ld + j0 + j] = a[i][j];
  }
}

// Rows [r0, r0 + nr) of X, columns [c0, c0 + w): x K^T = y with K the lower
// w x w block at (kb, kb) of Kf (ldk), solved row by row (one thread a row,
// the block in LDS).
__global__ __launch_bounds__(256) void cd_rowsolve_kernel(double *__restrict__ X, int64_t ldx, int64_t r0,
                                                          int64_t nr, int c0, int w,
                                                          const double *__restrict__ Kf, int ldk, int kb) {
  __shared__ double kk[64][65];
  const int tid = threadIdx.x;
  for (int e = tid; e < w * w; e += 256) {
    const int i = e / w, j = e - (e / w) * w;
    kk[i][j] = j <= i ? Kf[int64_t(kb + i) * ldk + kb + j] : 0.0;
  }
  __syncthreads();
  const int64_t r = r0 + int64_t(blockIdx.x) * 256 + tid;
  if (r >= r0 + nr) return;
  double *__restrict__ x = X + r * ldx + c0;
  double v[64];
#pragma unroll
  for (int j = 0; j < 64; ++j) v[j] = j < w ? x[j] : 0.0;
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    if (j < w) {
      double s = v[j];
#pragma unroll
      for (int i = 0; i < j; ++i) s -= v[i] * kk[j][i];
      v[j] = s / kk[j][j];
    }
  }
#pragma unroll
  for (int j = 0; j < 64; ++j)
    if (j < w) x[j] = v[j];
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_cd_diag(const double *V, int64_t n, double *D, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  cd_diag_kernel<<<int((n + 255) / 256), 256, 0, s>>>(V, n, D);
  return hipGetLastError();
}

hipError_t launch_cd_gather_cols(const double *V, int64_t n, const int32_t *qrows, int nq, double *M, int ldm,
                                 hipStream_t s) {
  if (n <= 0 || nq <= 0) return hipSuccess;
  cd_gather_cols_kernel<<<int((n * nq + 255) / 256), 256, 0, s>>>(V, n, qrows, nq, M, ldm);
  return hipGetLastError();
}

hipError_t launch_cd_micro(const CdQ *q, int nq, const CdPtrs &P, int64_t nmax, CdState *st, int steps,
                           hipStream_t s) {
  for (int t = 0; t < steps; ++t) {
    cd_argmax_kernel<<<1, 1024, 0, s>>>(q, nq, P, st);
    cd_column_kernel<<<int((nmax + 255) / 256), 256, 0, s>>>(P, st);
  }
  return hipGetLastError();
}

hipError_t launch_cd_gemm_nt(const CdGemm &G, hipStream_t s) {
  if (G.M <= 0 || G.N <= 0) return hipSuccess;
  dim3 grid((G.N + 63) / 64, (G.M + 63) / 64);
  cd_gemm_nt_kernel<<<grid, 256, 0, s>>>(G);
  return hipGetLastError();
}

hipError_t launch_cd_gather_metric(const double *V, int64_t n, const int32_t *piv, int np, double *K, double *Y,
                                   hipStream_t s) {
  const int64_t tot = int64_t(np) * np + n * np;
  if (tot <= 0) return hipSuccess;
  cd_gather_metric_kernel<<<int((tot + 255) / 256), 256, 0, s>>>(V, n, piv, np, K, Y);
  return hipGetLastError();
}

hipError_t launch_cd_potrf_diag(double *K, int ld, int j0, int w, int *bad, hipStream_t s) {
  cd_potrf_diag_kernel<<<1, 256, 0, s>>>(K, ld, j0, w, bad);
  return hipGetLastError();
}

hipError_t launch_cd_rowsolve(double *X, int64_t ldx, int64_t r0, int64_t nr, int c0, int w, const double *K,
                              int ldk, int kb, hipStream_t s) {
  if (nr <= 0 || w <= 0) return hipSuccess;
  cd_rowsolve_kernel<<<int((nr + 255) / 256), 256, 0, s>>>(X, ldx, r0, nr, c0, w, K, ldk, kb);
  return hipGetLastError();
}

}  // namespace cdcc
