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
// First step, per macro iteration (host loop in cdcc.cpp, cdcc_cd_basis):
//   gather     M[r][slot] = V[r][q_slot] for the qualified pairs q of an irrep
//   gemm_nt    M -= L1 L1[Q]^T (the vectors of earlier macro iterations)
//   micro      one launch per micro iteration: pivot = the first largest
//              Diag over Q, then the new vector over P, (M[r][q] - sum_mic
//              L1[r] L1[q]) / sqrt(d), and Diag(r) -= L^2; launched in chunks
//              without host synchronisation (a device flag ends them)
// Second step, per irrep: gather the metric V[piv][piv] and Y = V[:, piv];
// blocked right-looking Cholesky of the metric (64 x 64 diagonal block and its
// inverse in one wave; panel = panel Kinv^T and the trailing update as
// gemm_nt); then Y K^-T by 64-column blocks (gemm_nt update with the solved
// columns, then the block times Kinv^T): L[r][P].
#include <hip/hip_runtime.h>

#include <algorithm>

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

// One micro iteration of every irrep, fused (grid.y = irrep g): every
// workgroup of irrep g finds that irrep's pivot (the first largest diagonal
// over g's qualified pairs in Q order, from this step's copy dq_in of the
// qualified diagonals, which no workgroup writes during the step), and the
// workgroups of g together compute the new vector over the rows of g, 16
// lanes per row (partial dot products over the vectors of this macro
// iteration, combined by shuffles): L_r = (M[r][slot] - sum_mic L1[r] L1[q])
// / sqrt(d), Diag(r) -= L_r^2 (the pivot's own diagonal set to 0).  The next
// step's qualified diagonals of g go to dq_out and g's fields of the next
// state to st[par ^ 1]; workgroup 0 of g writes them and the pivot.  A
// largest value below tau_mic (or g's list used up) ends irrep g; later steps
// only carry its fields forward.  A step of g changes only g's diagonals, so
// running the irreps side by side gives each irrep the pivot sequence of the
// one-pivot-at-a-time loop.  Everything a row needs that does not depend on
// the pivot (membership, diagonal, slot and its first 256 entries of this
// macro iteration's vectors) is loaded before the pivot search, so a step
// has two dependent rounds of loads: state, diagonals and row data; then
// the pivot's row and residual column.
__global__ __launch_bounds__(256) void cd_micro_kernel(const int32_t *__restrict__ qr, CdQList QL, CdPtrs P,
                                                       CdState *__restrict__ st, int par,
                                                       const double *__restrict__ dq_in,
                                                       double *__restrict__ dq_out) {
  __shared__ double wv[4];
  __shared__ int wi[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = blockIdx.y;
  const CdState *S = st + par;
  CdState *__restrict__ nx = st + (par ^ 1);
  const int col = S->k[g], steps = S->steps[g];
  const bool lead = blockIdx.x == 0 && tid == 0;
  if (S->gdone[g]) {
    if (lead) {
      nx->k[g] = col;
      nx->gdone[g] = 1;
      nx->steps[g] = steps;
    }
    return;
  }
  const int beg = QL.beg[g], nqg = QL.cnt[g];
  const int k0 = S->k0[g];
  const int64_t n = P.n[g];
  const int nm = col - k0;
  double *__restrict__ L1 = P.L1[g];
  const int64_t r = (int64_t(blockIdx.x) * 256 + tid) >> 4;
  const int sub = tid & 15;
  const bool live = r < n;
  // row data that does not depend on the pivot, in flight during the search
  constexpr int kPre = 16;  // entries per lane held in registers (nm <= 256)
  int inp = 0, e2 = -1;
  double dr = 0.0, lrv[kPre];
  const CDCC_GLOBAL double *lr = as_global(L1) + (live ? r : 0) * n + k0;
  if (live) {
    inp = P.inP[g][r];
    dr = P.D[g][r];
    e2 = P.qpos[g][r];
  }
#pragma unroll
  for (int t = 0; t < kPre; ++t) {
    const int i = sub + 16 * t;
    lrv[t] = (live && i < nm) ? lr[i] : 0.0;
  }
  // pivot: first maximum in Q order among g's entries
  double best = -__builtin_huge_val();
  int bi = nqg;
  for (int e = tid; e < nqg; e += 256) {
    const double v = dq_in[beg + e];
    if (v > best) {
      best = v;
      bi = e;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const double v2 = __shfl_xor(best, o);
    const int i2 = __shfl_xor(bi, o);
    if (v2 > best || (v2 == best && i2 < bi)) {
      best = v2;
      bi = i2;
    }
  }
  if (lane == 0) {
    wv[wave] = best;
    wi[wave] = bi;
  }
  __syncthreads();
  best = wv[0];
  bi = wi[0];
  for (int w = 1; w < 4; ++w)
    if (wv[w] > best || (wv[w] == best && wi[w] < bi)) {
      best = wv[w];
      bi = wi[w];
    }
  if (bi >= nqg || !(best >= S->tau_mic) || steps >= nqg) {
    if (lead) {
      nx->k[g] = col;
      nx->gdone[g] = 1;
      nx->steps[g] = steps;
    }
    return;
  }
  const int prow = qr[beg + bi];
  if (lead) {
    nx->k[g] = col + 1;
    nx->gdone[g] = 0;
    nx->steps[g] = steps + 1;
    P.piv[g][col] = prow;
  }
  if (!live) return;  // whole 16-lane groups leave together
  if (!inp) {
    if (sub == 0) L1[r * n + col] = 0.0;
    return;
  }
  const double m = P.M[g][r * P.qcap[g] + bi];
  const CDCC_GLOBAL double *lq = as_global(L1) + int64_t(prow) * n + k0;
  double a = 0.0;
#pragma unroll
  for (int t = 0; t < kPre; ++t) {
    const int i = sub + 16 * t;
    a += lrv[t] * (i < nm ? lq[i] : 0.0);
  }
  for (int i = sub + 16 * kPre; i < nm; i += 16) a += lr[i] * lq[i];
  a += __shfl_xor(a, 8);
  a += __shfl_xor(a, 4);
  a += __shfl_xor(a, 2);
  a += __shfl_xor(a, 1);
  if (sub == 0) {
    const double v = (m - a) / sqrt(best);
    L1[r * n + col] = v;
    const double dn = (r == prow) ? 0.0 : dr - v * v;
    P.D[g][r] = dn;
    if (e2 >= 0) dq_out[beg + e2] = dn;
  }
}

// ---------------------------------------------------------------------------
// generic C[m][n] = beta C[m][n] + alpha sum_k A[arow(m)][k] B[brow(n)][k]
// (C not read when beta = 0; both operands
// K-contiguous rows; optional row-index tables), 64 x 64 tiles, 4 waves in
// 2 x 2 of MFMA f64 16x16x4, BK = 16 double-buffered LDS ([k][m], [k][n]).
// Rows past M / N read a clamped row and are not stored; k past K is zeroed
// by a select.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cd_gemm_nt_kernel(CdGemmBatch GB) {
  constexpr int BM = 64, BK = 16, LD = BM + 2;
  __shared__ double As[2][BK][LD], Bs[2][BK][LD];
  const CdGemm &G = GB.g[blockIdx.z];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BM;
  if (m0 >= G.M || n0 >= G.N) return;  // the grid covers the largest GEMM of the batch
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
          *c = G.beta == 0.0 ? G.alpha * acc[i][j][r] : G.beta * *c + G.alpha * acc[i][j][r];
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

// Lower Cholesky factor of the w x w block at (j0, j0) of K (ld), in place,
// and its inverse into Kinv (64 x 64, row-major, zero above the diagonal and
// outside w), one workgroup per irrep of the batch; a non-positive pivot
// sets *bad.  One wave: lane i holds row i
// of the block in registers (factor), then column i of the inverse (forward
// substitution against the factor, read from LDS).
__global__ __launch_bounds__(64) void cd_potrf_diag_kernel(CdDiagBatch DB, int *__restrict__ bad) {
  __shared__ double lf[64][65];
  __shared__ double piv_s;
  double *__restrict__ K = DB.K[blockIdx.x];
  double *__restrict__ Kinv = DB.Kinv[blockIdx.x];
  const int ld = DB.ld[blockIdx.x], j0 = DB.j0[blockIdx.x], w = DB.w[blockIdx.x];
  const int i = threadIdx.x;
  double a[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) a[k] = (i < w && k <= i && k < w) ? K[int64_t(j0 + i) * ld + j0 + k] : 0.0;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    if (j < w) {
      if (i == j) piv_s = a[j];
      __syncthreads();
      const double d = piv_s;
      ok = ok && (d > 0.0);
      const double sd = sqrt(d > 0.0 ? d : 1.0);
      const double lij = (i > j) ? a[j] / sd : (i == j ? sd : 0.0);
      a[j] = lij;
      lf[i][j] = lij;
      __syncthreads();
      // every lane updates its whole row: entries above its diagonal or past
      // w collect values that are never read (lij = 0 for i < j, lf = 0
      // past w), which keeps the loop free of lane-dependent branches
#pragma unroll
      for (int k = j + 1; k < 64; ++k) a[k] -= lij * lf[k][j];
    }
  }
  if (i == 0 && !ok) *bad = 1;
  if (i < w) {
#pragma unroll
    for (int k = 0; k < 64; ++k)
      if (k <= i && k < w) K[int64_t(j0 + i) * ld + j0 + k] = a[k];
  }
  // inverse: lane c solves L x = e_c (x = column c of L^-1)
  double x[64];
#pragma unroll
  for (int r = 0; r < 64; ++r) {
    double t = (r == i) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < r; ++k) t -= lf[r][k] * x[k];
    x[r] = (r < w && i < w && r >= i) ? t / lf[r][r] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < 64; ++r) Kinv[r * 64 + i] = x[r];
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

hipError_t launch_cd_micro(const int32_t *qr, const CdQList &QL, const CdPtrs &P, int64_t nmax, int nirrep,
                           CdState *st, double *dq, int qcap, int t0, int steps, hipStream_t s) {
  const dim3 grid(unsigned(std::max<int64_t>((nmax * 16 + 255) / 256, 1)), unsigned(nirrep));
  for (int t = t0; t < t0 + steps; ++t) {
    const int par = t & 1;
    cd_micro_kernel<<<grid, 256, 0, s>>>(qr, QL, P, st, par, dq + par * qcap, dq + (par ^ 1) * qcap);
  }
  return hipGetLastError();
}

hipError_t launch_cd_gemm_nt(const CdGemmBatch &B, hipStream_t s) {
  int mm = 0, nn = 0;
  for (int k = 0; k < B.n; ++k) {
    mm = std::max(mm, B.g[k].M);
    nn = std::max(nn, B.g[k].N);
  }
  if (B.n <= 0 || mm <= 0 || nn <= 0) return hipSuccess;
  dim3 grid((nn + 63) / 64, (mm + 63) / 64, B.n);
  cd_gemm_nt_kernel<<<grid, 256, 0, s>>>(B);
  return hipGetLastError();
}

hipError_t launch_cd_gather_metric(const double *V, int64_t n, const int32_t *piv, int np, double *K, double *Y,
                                   hipStream_t s) {
  const int64_t tot = int64_t(np) * np + n * np;
  if (tot <= 0) return hipSuccess;
  cd_gather_metric_kernel<<<int((tot + 255) / 256), 256, 0, s>>>(V, n, piv, np, K, Y);
  return hipGetLastError();
}

hipError_t launch_cd_potrf_diag(const CdDiagBatch &D, int *bad, hipStream_t s) {
  if (D.n <= 0) return hipSuccess;
  cd_potrf_diag_kernel<<<D.n, 64, 0, s>>>(D, bad);
  return hipGetLastError();
}

}  // namespace cdcc
