// O(O^3 V^3) contraction with the partial symmetric-antisymmetric algorithm,
// FP64 kernels for gfx950 (CDNA4).
//
// Paper: the paragraph closing the section on the spin-adapted I_pq
// multipliers (the symmetric-antisymmetric algorithm for the O(O^2 V^4)
// terms and its partial variant for the O(O^3 V^3) ones, example
// M_bi^dc = sum_mn lambda_Bi^Mn tau~_mn^dc).  Only lambda's (m, n) pair can be
// folded; tau~ is pair symmetric, so tau+/- are symmetric/antisymmetric in
// (d, c) and only the d >= c columns are computed:
//
//   lam+ = lam_bi^mn + lam_bi^nm (m > n), lam_bi^mm;   lam- = lam_bi^mn - lam_bi^nm
//   tau+ = tau_mn^dc + tau_mn^cd;                       tau- = tau_mn^dc - tau_mn^cd
//   S = sum_{m>=n} lam+ tau+,  A = sum_{m>=n} lam- tau-  (lam- = 0 for m = n)
//   M_bi^dc = (S + A) / 2,     M_bi^cd = (S - A) / 2
//
// Pipeline of one call (all systems and pair irreps in each launch):
//   pack_lam  lam+/- rows (b,i), K = the m >= n pairs, zero-padded to 16
//   pack_tau  tau+/- rows m >= n, columns grouped in squares of 8 d x 8 c
//   gemm      one 64-row x one-square tile of S and A per workgroup (MFMA
//             f64), then M_bi^dc from registers and M_bi^cd through LDS
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"

namespace cdcc {

typedef double pd2 __attribute__((ext_vector_type(2)));
typedef double pd4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// lam+/- : one thread per (row, k) element of [nrow][ldk]; rows are read
// from the lambda block (each row n_oo contiguous doubles, cached).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pm_pack_lam_kernel(const PmDesc *__restrict__ descs,
                                                          const PmChunk *__restrict__ chunks,
                                                          const int2 *__restrict__ kp,
                                                          const PmPtrs *__restrict__ pp) {
  const PmChunk c = chunks[blockIdx.x];
  const PmDesc D = descs[c.desc];
  const int64_t n = int64_t(D.nrow) * D.ldk;
  const int64_t e = int64_t(c.chunk) * 256 + threadIdx.x;
  if (e >= n) return;
  const PmPtrs P = pp[D.sys];
  const int row = int(e / D.ldk), k = int(e - int64_t(row) * D.ldk);
  double vp = 0.0, vm = 0.0;
  if (k < D.nk) {
    const int2 q = kp[D.kp_off + k];
    const CDCC_GLOBAL double *lr = as_global(P.lam) + D.lam_off + int64_t(row) * D.n_oo;
    const double x = lr[q.x];
    if (q.x == q.y) {
      vp = x;
    } else {
      const double y = lr[q.y];
      vp = x + y;
      vm = x - y;
    }
  }
  double *__restrict__ lp = P.ws + D.lp_off;
  lp[e] = vp;
  lp[n + e] = vm;
}

// ---------------------------------------------------------------------------
// tau+/- : one thread per (k, column) element of [ldk][nsq * 64]; column
// w of a square is (dd, cc) = (w / 8, w % 8).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pm_pack_tau_kernel(const PmDesc *__restrict__ descs,
                                                          const PmChunk *__restrict__ chunks,
                                                          const int2 *__restrict__ kp,
                                                          const PmSquare *__restrict__ sqs,
                                                          const PmPtrs *__restrict__ pp) {
  const PmChunk c = chunks[blockIdx.x];
  const PmDesc D = descs[c.desc];
  const int ncol = D.nsq * 64;
  const int64_t n = int64_t(D.ldk) * ncol;
  const int64_t e = int64_t(c.chunk) * 256 + threadIdx.x;
  if (e >= n) return;
  const PmPtrs P = pp[D.sys];
  const int k = int(e / ncol), col = int(e - int64_t(k) * ncol);
  const PmSquare Q = sqs[D.sq_off + (col >> 6)];
  const int dd = (col >> 3) & 7, cc = col & 7;
  double vp = 0.0, vm = 0.0;
  if (k < D.nk && dd < Q.nd && cc < Q.nc) {
    const int2 q = kp[D.kp_off + k];
    const CDCC_GLOBAL double *tr = as_global(P.tau) + D.tau_off + int64_t(q.x) * D.n_vv;
    const double a = tr[Q.base_dc + dd * Q.ld_dc + cc];
    const double b = tr[Q.base_cd + cc * Q.ld_cd + dd];
    vp = a + b;
    vm = a - b;
  }
  double *__restrict__ tp = P.ws + D.tp_off;
  tp[e] = vp;
  tp[n + e] = vm;
}

// ---------------------------------------------------------------------------
// gemm: one workgroup per (block, 64-row tile, square); 4 waves in 2 x 2,
// each 32 x 32 of both S and A (MFMA f64 16x16x4); BK = 8 double-buffered
// LDS stages of lam+, lam- (transposed to [k][m]) and tau+, tau- ([k][n]).
// K is zero-padded to a multiple of 16, rows past nrow read a clamped row
// (not stored).  Epilogue: M_bi^dc straight from the accumulators (the 16
// lanes of a row hold two 8-wide (d, c) runs), and off the block diagonal
// M_bi^cd through a transposing pass in LDS (dd fastest).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 3) void pm_gemm_kernel(const PmDesc *__restrict__ descs,
                                                         const int4 *__restrict__ tiles,
                                                         const PmSquare *__restrict__ sqs,
                                                         const PmPtrs *__restrict__ pp) {
  constexpr int BM = 64, BK = 8, LD = BM + 2, LE = 65;
  __shared__ double lds[2][4][BK][LD];  // [buffer][lam+, lam-, tau+, tau-][k][m or n]
  static_assert(sizeof(lds) >= BM * LE * sizeof(double), "epilogue reuses the staging buffer");

  const int4 tl = tiles[blockIdx.x];
  const PmDesc D = descs[tl.x];
  const PmPtrs P = pp[D.sys];
  const PmSquare Q = sqs[D.sq_off + tl.z];
  const int m0 = tl.y * BM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int ncol = D.nsq * 64;

  const int ar = tid >> 2, ak = (tid & 3) * 2;     // A staging: row, 2 k
  const int bk = tid >> 5, bn = (tid & 31) * 2;    // B staging: k, 2 columns
  const CDCC_GLOBAL double *lp =
      as_global(P.ws) + D.lp_off + int64_t(min(m0 + ar, D.nrow - 1)) * D.ldk + ak;
  const CDCC_GLOBAL double *lm = lp + int64_t(D.nrow) * D.ldk;
  const CDCC_GLOBAL double *tp = as_global(P.ws) + D.tp_off + int64_t(bk) * ncol + tl.z * 64 + bn;
  const CDCC_GLOBAL double *tm = tp + int64_t(D.ldk) * ncol;

  pd4 accS[2][2], accA[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accS[i][j] = pd4{0.0, 0.0, 0.0, 0.0};
      accA[i][j] = pd4{0.0, 0.0, 0.0, 0.0};
    }

  pd2 ra[2], rb[2];
  auto gload = [&](int k0) {
    ra[0] = *reinterpret_cast<const CDCC_GLOBAL pd2 *>(lp + k0);
    ra[1] = *reinterpret_cast<const CDCC_GLOBAL pd2 *>(lm + k0);
    rb[0] = *reinterpret_cast<const CDCC_GLOBAL pd2 *>(tp + int64_t(k0) * ncol);
    rb[1] = *reinterpret_cast<const CDCC_GLOBAL pd2 *>(tm + int64_t(k0) * ncol);
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      lds[buf][s][ak + 0][ar] = ra[s].x;
      lds[buf][s][ak + 1][ar] = ra[s].y;
      lds[buf][2 + s][bk][bn + 0] = rb[s].x;
      lds[buf][2 + s][bk][bn + 1] = rb[s].y;
    }
  };

  const int nkb = D.ldk / BK;
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
      double fap[2], fam[2], fbp[2], fbm[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        fap[i] = lds[cur][0][kr][wm * 32 + i * 16 + (lane & 15)];
        fam[i] = lds[cur][1][kr][wm * 32 + i * 16 + (lane & 15)];
        fbp[i] = lds[cur][2][kr][wn * 32 + i * 16 + (lane & 15)];
        fbm[i] = lds[cur][3][kr][wn * 32 + i * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          accS[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fap[i], fbp[j], accS[i][j], 0, 0, 0);
          accA[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fam[i], fbm[j], accA[i][j], 0, 0, 0);
        }
    }
    if (more) lstore(cur ^ 1);
    __syncthreads();
  }

  double *__restrict__ Mb = P.M + D.m_off;
  // M_bi^dc from the accumulators: tile column w = dd * 8 + cc
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int w = wn * 32 + j * 16 + (lane & 15);
      const int dd = w >> 3, cc = w & 7;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * r;
        if (row < D.nrow && dd < Q.nd && cc < Q.nc)
          Mb[int64_t(row) * D.n_vv + Q.base_dc + dd * Q.ld_dc + cc] = 0.5 * (accS[i][j][r] + accA[i][j][r]);
      }
    }
  if (Q.diag) return;  // uniform: the square holds both orders
  // M_bi^cd: (S - A) / 2 through LDS (the staging buffer is free after the
  // last barrier of the K loop), then dd-fastest runs
  double(*sD)[LE] = reinterpret_cast<double(*)[LE]>(&lds[0][0][0][0]);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        sD[wm * 32 + i * 16 + (lane >> 4) + 4 * r][wn * 32 + j * 16 + (lane & 15)] =
            0.5 * (accS[i][j][r] - accA[i][j][r]);
  __syncthreads();
  for (int e = tid; e < BM * 64; e += 256) {
    const int dd = e & 7, cc = (e >> 3) & 7, r = e >> 6;
    const int row = m0 + r;
    if (row >= D.nrow || dd >= Q.nd || cc >= Q.nc) continue;
    Mb[int64_t(row) * D.n_vv + Q.base_cd + cc * Q.ld_cd + dd] = sD[r][dd * 8 + cc];
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_pm_pack(const PmDesc *descs, const PmChunk *lch, int nl, const PmChunk *tch, int nt,
                          const int2 *kp, const PmSquare *sqs, const PmPtrs *pp, hipStream_t s) {
  if (nl > 0) pm_pack_lam_kernel<<<nl, 256, 0, s>>>(descs, lch, kp, pp);
  if (nt > 0) pm_pack_tau_kernel<<<nt, 256, 0, s>>>(descs, tch, kp, sqs, pp);
  return hipGetLastError();
}

hipError_t launch_pm_gemm(const PmDesc *descs, const int4 *tiles, int ntiles, const PmSquare *sqs,
                          const PmPtrs *pp, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  pm_gemm_kernel<<<ntiles, 256, 0, s>>>(descs, tiles, sqs, pp);
  return hipGetLastError();
}

}  // namespace cdcc
