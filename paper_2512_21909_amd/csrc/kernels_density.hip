// vvvv block of the spin-adapted CCSD two-body density contracted with
// Cholesky vectors, FP64 kernels for gfx950 (CDNA4).
//
// Paper: Appendix "CCSD two-body density matrices" (Gamma_AbCd =
// 1/2 P_+(ab,cd) V_AbCd, V_AbEf = sum_mn tau_Mn^Ef lambda_Ab^Mn), the
// spin-adapted density Gamma~_pqrs = 2 Gamma_PqRs - Gamma_PqSr of the section
// on CCSD density matrices, and the gradient section (Gamma^P_pr = sum_qs
// Gamma~_pqrs L~^P_qs, contracted on the fly).  Closed-shell spatial form
// computed here, with X = tau~, Y = lambda and X'^cd = 2 X^cd - X^dc,
// Y'^cd = 2 Y^cd - Y^dc:
//
//   W_(ab),(cd) = sum_mn [Y_mn^ab X'_mn^cd + X_mn^ab Y'_mn^cd]  = 2 Gamma~_abcd
//   G^P_ac      = 1/2 sum_bd W_(ab),(cd) L^P_bd
//
// (2 Gamma~_abcd = sum_mn [Y^ab (2X^cd - X^dc) + X^ab (2Y^cd - Y^dc)]: the
// P_+ pair of V_abcd and V_cdab, minus half the pair of V_abdc and V_dcab.)
//
// Pipeline of one call:
//   pack   amplitude blocks (rows mn, columns ab) -> T tables, rows (ab) of
//          [Y | X] and rows (cd) of [X' | Y'] (K = 2 n_oo(G), contiguous), so
//          W is one GEMM T T'^T with K = 2 n_oo (the assembly kernel, mode 1,
//          writes W with rows (a, c) and columns (b, d) into a bounded batch
//          buffer)
//   gemm   G[(a,c)][P] = 1/2 W[(a,c)][(b,d)] L[(b,d)][P] over the (b, d) pairs
//          of the Cholesky irrep (below), K cut into fixed segments
//   reduce partial tiles of the segments summed in segment order
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"

namespace cdcc {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// pack: one workgroup per 64 x 64 tile (64 mn rows x 64 columns) of one
// (system, G) amplitude block; read along the columns, written along mn
// through LDS, in two passes: [Y | X] for the rows (ab), then [X' | Y'] for
// the rows (cd), whose exchange partners X^dc, Y^dc are read at the swapped
// column of the same mn row (swap table of the job).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void density_pack_kernel(const DensPackJob *__restrict__ jobs,
                                                           const int2 *__restrict__ tiles,
                                                           const int *__restrict__ swap,
                                                           const DensPtrs *__restrict__ dp) {
  __shared__ double ly[64][65], lx[64][65];
  const int2 jt = tiles[blockIdx.x];
  const DensPackJob J = jobs[jt.x];
  const DensPtrs P = dp[J.sys];
  const int ncb = (J.ncol + 63) / 64;
  const int k0 = (jt.y / ncb) * 64, c0 = (jt.y % ncb) * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const CDCC_GLOBAL double *y = as_global(P.Y) + J.x_off;
  const CDCC_GLOBAL double *x = as_global(P.X) + J.x_off;
  const int c = c0 + tx;
  const bool cin = c < J.ncol;
  const int csw = cin ? swap[J.sw_off + c] : 0;
  const int K2 = 2 * J.nrow;
  double *__restrict__ tw = P.T + J.tw_off;                  // [Y | X]
  double *__restrict__ tv = tw + int64_t(J.ncol) * K2;       // [X' | Y']
  const int k = k0 + tx;
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int kk = ty + 4 * q, kr = k0 + kk;
      const bool in = kr < J.nrow && cin;
      const int64_t row = int64_t(in ? kr : 0) * J.ncol;
      const int64_t o = row + (in ? c : 0);
      double yv = y[o], xv = x[o];
      if (pass == 1) {
        const int64_t os = row + (in ? csw : 0);
        yv = 2.0 * yv - y[os];
        xv = 2.0 * xv - x[os];
      }
      ly[kk][tx] = in ? yv : 0.0;
      lx[kk][tx] = in ? xv : 0.0;
    }
    __syncthreads();
    double *__restrict__ tt = pass == 0 ? tw : tv;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int cc = ty + 4 * q, col = c0 + cc;
      if (k >= J.nrow || col >= J.ncol) continue;
      const int64_t r = int64_t(col) * K2;
      tt[r + k] = pass == 0 ? ly[tx][cc] : lx[tx][cc];
      tt[r + J.nrow + k] = pass == 0 ? lx[tx][cc] : ly[tx][cc];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// gemm (second stage), persistent: one work unit = one BM x BN tile of one K
// segment.  BK = 16, 4 waves in 2 x 2, MFMA f64 16x16x4.  A rows
// (K-contiguous, lda a multiple of 4) are read 4 k at a time and staged
// transposed into LDS [k][m]; B rows ([k][n], n-contiguous) are staged as
// they are; double buffered, one barrier per K step.  Rows past M and columns
// past N are read from clamped addresses and their results are not stored;
// k past the segment end (last block only) reads a clamped address and is
// zeroed by a select, so padding columns of A are never read.
// ---------------------------------------------------------------------------
template <int BM, int BN>
__global__ __launch_bounds__(256, 2) void gemm_nn_f64_kernel(const GemmDesc *__restrict__ descs,
                                                             const Tile *__restrict__ tiles, Queues Q,
                                                             int *__restrict__ cnt,
                                                             const DensPtrs *__restrict__ dp,
                                                             const double *__restrict__ xbuf,
                                                             double *__restrict__ part) {
  constexpr int BK = 16;
  constexpr int LA = BM + 2, LB = BN + 2;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int RA = BM / 64;              // A rows per thread (4 consecutive k each)
  constexpr int CB = BN * BK / 256;        // B columns per thread (one k row)
  constexpr int TPK = BN / CB;             // threads per B k row
  static_assert(CB >= 1 && 256 / TPK == BK, "B staging");
  __shared__ double As[2][BK][LA];
  __shared__ double Bs[2][BK][LB];
  __shared__ int s_tile;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = tid >> 2, lk = (tid & 3) * 4;   // A staging
  const int bk = tid / TPK, bc = (tid % TPK) * CB;  // B staging
  unsigned dead = 0;

  for (;;) {
    const int t = next_tile(cnt, Q, dead, &s_tile);
    if (t < 0) break;
    const Tile tl = tiles[t];
    const GemmDesc D = descs[tl.desc];
    const DensPtrs P = dp[D.sys];
    const int m0 = tl.tm * BM, n0 = tl.tn * BN;
    const int kseg0 = tl.aux * kGemmKSeg;
    const int K = min(D.K - kseg0, kGemmKSeg);
    const CDCC_GLOBAL double *arow[RA];
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int m = min(m0 + lr + 64 * q, D.M - 1);
      arow[q] = as_global(xbuf) + D.aoff + int64_t(m) * D.lda + kseg0 + lk;
    }
    const CDCC_GLOBAL double *brow = as_global(P.L) + D.boff + int64_t(kseg0 + bk) * D.ldb;
    int bcol[CB];
#pragma unroll
    for (int e = 0; e < CB; ++e) bcol[e] = min(n0 + bc + e, D.N - 1);

    d4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    double ra[RA][4], rb[CB];
    auto gload = [&](int k0) {  // a whole block
#pragma unroll
      for (int q = 0; q < RA; ++q) {
        const CDCC_GLOBAL d2 *pa = reinterpret_cast<const CDCC_GLOBAL d2 *>(arow[q] + k0);
        const d2 u = pa[0], v = pa[1];
        ra[q][0] = u.x;
        ra[q][1] = u.y;
        ra[q][2] = v.x;
        ra[q][3] = v.y;
      }
      const CDCC_GLOBAL double *br = brow + int64_t(k0) * D.ldb;
#pragma unroll
      for (int e = 0; e < CB; ++e) rb[e] = br[bcol[e]];
    };
    auto gload_tail = [&](int k0) {  // the last, partial block
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = k0 + lk + e;
        const int kc = min(k, K - 1) - lk;
#pragma unroll
        for (int q = 0; q < RA; ++q) {
          const double x = arow[q][kc];
          ra[q][e] = k < K ? x : 0.0;
        }
      }
      const int k = k0 + bk;
      const CDCC_GLOBAL double *br = brow + int64_t(min(k, K - 1) - bk) * D.ldb;
#pragma unroll
      for (int e = 0; e < CB; ++e) {
        const double x = br[bcol[e]];
        rb[e] = k < K ? x : 0.0;
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int q = 0; q < RA; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) As[buf][lk + e][lr + 64 * q] = ra[q][e];
#pragma unroll
      for (int e = 0; e < CB; ++e) Bs[buf][bk][bc + e] = rb[e];
    };

    const int nfull = K / BK, nk = (K + BK - 1) / BK;
    if (nfull > 0) gload(0);
    else gload_tail(0);
    lstore(0);
    __syncthreads();
    for (int kb = 0; kb < nk; ++kb) {
      const int cur = kb & 1, kn = kb + 1;
      if (kn < nfull) gload(kn * BK);
      else if (kn < nk) gload_tail(kn * BK);
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        const int kr = ks * 4 + (lane >> 4);
        double fa[FM], fb[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) fa[i] = As[cur][kr][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < FN; ++j) fb[j] = Bs[cur][kr][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
      }
      if (kn < nk) lstore(cur ^ 1);
      __syncthreads();
    }

    if (D.nseg == 1) {
      double *__restrict__ C = P.G + D.coff;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int m = m0 + wm * WM + i * 16 + (lane >> 4) + 4 * r;
            const int n = n0 + wn * WN + j * 16 + (lane & 15);
            if (m >= D.M || n >= D.N) continue;
            C[int64_t(m) * D.ldc + n] = D.alpha * acc[i][j][r];
          }
    } else {
      double *__restrict__ pb =
          part + D.poff + (int64_t(tl.tm * D.tiles_n + tl.tn) * D.nseg + tl.aux) * (BM * BN);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int lm = wm * WM + i * 16 + (lane >> 4) + 4 * r;
            const int ln = wn * WN + j * 16 + (lane & 15);
            pb[lm * BN + ln] = acc[i][j][r];
          }
    }
  }
}

// ---------------------------------------------------------------------------
// reduce (split K): one workgroup per output tile; the partial tiles are
// summed in segment order, scaled by alpha and stored.
// ---------------------------------------------------------------------------
template <int BM, int BN>
__global__ __launch_bounds__(256) void gemm_reduce_kernel(const GemmDesc *__restrict__ descs,
                                                          const Tile *__restrict__ jobs,
                                                          const DensPtrs *__restrict__ dp,
                                                          const double *__restrict__ part) {
  const Tile tl = jobs[blockIdx.x];
  const GemmDesc D = descs[tl.desc];
  double *__restrict__ C = dp[D.sys].G + D.coff;
  const CDCC_GLOBAL double *pb =
      as_global(part) + D.poff + int64_t(tl.tm * D.tiles_n + tl.tn) * D.nseg * (BM * BN);
#pragma unroll 4
  for (int e = threadIdx.x; e < BM * BN; e += 256) {
    const int m = tl.tm * BM + e / BN, n = tl.tn * BN + e % BN;
    if (m >= D.M || n >= D.N) continue;
    double s = pb[e];
    for (int k = 1; k < D.nseg; ++k) s += pb[int64_t(k) * (BM * BN) + e];
    C[int64_t(m) * D.ldc + n] = D.alpha * s;
  }
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_density_pack(const DensPackJob *jobs, const int2 *tiles, int ntiles, const int *swap,
                               const DensPtrs *dp, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  density_pack_kernel<<<ntiles, 256, 0, s>>>(jobs, tiles, swap, dp);
  return hipGetLastError();
}

hipError_t launch_density_gemm(int grid, const GemmDesc *descs, const Tile *tiles, const Queues &Q, int *cnt,
                               const DensPtrs *dp, const double *xbuf, double *part, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  gemm_nn_f64_kernel<kGemmBM, kGemmBN><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, dp, xbuf, part);
  return hipGetLastError();
}

hipError_t launch_density_reduce(int njobs, const GemmDesc *descs, const Tile *jobs, const DensPtrs *dp,
                                 const double *part, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  gemm_reduce_kernel<kGemmBM, kGemmBN><<<njobs, 256, 0, s>>>(descs, jobs, dp, part);
  return hipGetLastError();
}

int occupancy_density_gemm() {
  int n = 0;
  const hipError_t e =
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, gemm_nn_f64_kernel<kGemmBM, kGemmBN>, 256, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace cdcc
