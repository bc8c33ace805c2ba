// FP64 kernels of the particle-particle ladder for gfx950 (CDNA4).
//
// Pipeline of one evaluation (paper: PPL equations of the Lambda section,
// symmetric-antisymmetric algorithm; Appendix A for the Lambda W):
//   pack     X -> tauhat(+/-), stored halves i>=j, c>=d, weights folded in
//   dress    (Lambda) U^P_ae = B^P_ea - t^P_ea and t^P_ea, a signed K stack
//   assemble X_{cd,ab} = 1/2 sum_P U^P_ac U^P_bd into a bounded batch buffer
//            (grouped GEMM on MFMA f64 16x16x4, operands staged in LDS)
//   contract S = tauhat(+) W(+), A = tauhat(-) W(-), W(+/-) = X_cd +/- X_dc
//            formed while staging; the epilogue unpacks S +/- A into the four
//            (ij,ab) permutations of R and writes R / D
//   energy   e_ij = sum_ab (2 X_ij^ab - X_ij^ba) R_ij^ab, fixed-order tree
// Tiles are pulled from per-XCD integer work queues by persistent workgroups.
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"

namespace cdcc {

typedef double d2 __attribute__((ext_vector_type(2)));
typedef double d4 __attribute__((ext_vector_type(4)));

// MFMA f64 16x16x4 lane mapping (gfx950): A[i][k] in lane i + 16k,
// B[k][j] in lane j + 16k, result register r of lane l is D[l/16 + 4r][l%16].

__global__ void fill_int_kernel(int *p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// pack: one workgroup per 64 x 64 tile of (packed row i>=j, packed column
// c>=d) of one (system, G).
//   tauhat(+)_ij^cd = X_ij^cd + X_ij^dc   (c>d),   X_ij^cc   (c=d)
//   tauhat(-)_ij^cd = X_ij^cd - X_ij^dc   (c>d),   0         (c=d or i=j)
// The halves are stored column-major (element (r, k) at k * ldt + r) for
// the contraction; the tile is read along rows of X and written along
// columns of tauhat through LDS, so both sides are coalesced.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pack_kernel(const PackJob *__restrict__ jobs,
                                                   const int2 *__restrict__ tiles,
                                                   const SysPtrs *__restrict__ sp,
                                                   const int4 *__restrict__ ijtab,
                                                   const int4 *__restrict__ vvtab) {
  __shared__ double lp[64][65], lm[64][65];
  const int2 jt = tiles[blockIdx.x];
  const PackJob J = jobs[jt.x];
  const int nkb = (J.ncol + 63) / 64;
  const int r0 = (jt.y / nkb) * 64, k0 = (jt.y % nkb) * 64;
  const SysPtrs S = sp[J.sys];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int k = k0 + tx;
  int4 cd = int4{0, 0, 0, 0};
  if (k < J.ncol) cd = vvtab[J.vv_off + k];
  const bool dcd = cd.x == cd.y;
  // all 16 rows of this thread: table entries first, then the amplitude
  // loads, then the arithmetic (clamped rows are computed and not stored)
  int2 ijr[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r = r0 + ty + 4 * q;
    const int4 ij = ijtab[J.ij_off + (r < J.nrow ? r : J.nrow - 1)];
    ijr[q] = int2{ij.x, ij.y};
  }
  double v1[16], v2[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const CDCC_GLOBAL double *xr = as_global(S.X) + J.x_off + int64_t(ijr[q].x) * J.ldx;
    v1[q] = xr[cd.x];
    v2[q] = xr[cd.y];
  }
  if (k < J.ncol) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int rr = ty + 4 * q;
      lp[rr][tx] = dcd ? v1[q] : v1[q] + v2[q];
      lm[rr][tx] = (dcd || ijr[q].x == ijr[q].y) ? 0.0 : v1[q] - v2[q];
    }
  }
  __syncthreads();
  double *__restrict__ tp = S.tauhat + J.th_off;
  double *__restrict__ tm = tp + int64_t(J.ldt) * J.ncol;
  const int r = r0 + tx;
  for (int kk = ty; kk < 64; kk += 4) {
    const int kc = k0 + kk;
    if (r >= J.nrow || kc >= J.ncol) continue;
    tp[int64_t(kc) * J.ldt + r] = lp[tx][kk];
    tm[int64_t(kc) * J.ldt + r] = lm[tx][kk];
  }
}

// ---------------------------------------------------------------------------
// dress (Lambda, Appendix A): one workgroup per (job, a, e), Ge = Ga^GP,
// threads along P:
//   t^P_ea = sum_m t_m^e L^P_am,  U[a][e][P] = B^P_ea - t^P_ea,
//   U[a][e][np + P] = t^P_ea   (subtracted in the assembly: kneg = np)
// Without singles only the first half is written (U = B transposed).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void dress_kernel(const DressJob *__restrict__ jobs,
                                                    const int2 *__restrict__ rows,
                                                    const SysPtrs *__restrict__ sp) {
  const int2 jr = rows[blockIdx.x];
  const DressJob J = jobs[jr.x];
  const int a = jr.y / J.ve, e = jr.y - a * J.ve;
  const SysPtrs S = sp[J.sys];
  double *__restrict__ U = const_cast<double *>(S.opnd);
  const bool dressed = S.t1 != nullptr && S.Bvo != nullptr;
  const int kst = dressed ? 2 * J.np : J.np;
  const CDCC_GLOBAL double *bea = as_global(S.B) + J.b_off + (int64_t(e) * J.va + a) * J.np;
  double *__restrict__ urow = U + J.u_off + (int64_t(a) * J.ve + e) * kst;
  if (!dressed) {
    for (int P = threadIdx.x; P < J.np; P += 256) urow[P] = bea[P];
    return;
  }
  const CDCC_GLOBAL double *lam = as_global(S.Bvo) + J.bvo_off + int64_t(a) * J.om * J.np;
  const CDCC_GLOBAL double *t1e = as_global(S.t1) + J.t1_off + e;
#pragma unroll 2
  for (int P = threadIdx.x; P < J.np; P += 256) {
    double tea = 0.0;
    for (int m = 0; m < J.om; ++m) tea += t1e[int64_t(m) * J.ve] * lam[int64_t(m) * J.np + P];
    urow[P] = bea[P] - tea;
    urow[J.np + P] = tea;
  }
}

// ---------------------------------------------------------------------------
// assemble (FP64): X[(c,d),(a,b)] = 1/2 sum_K U[(a,c),K] s_K U[(b,d),K]
// Tile BM x BN of the (a,c) x (d,b) product, BK = 16, 4 waves in 2x2, each
// wave (BM/2) x (BN/2) as 16x16 MFMA f64 blocks.  LDS holds [row][k] (rows
// of BK + 1 doubles, double-buffered, one barrier per K step).  Out-of-range rows
// and K are read from a clamped address and zeroed by a select, so the loads
// are straight-line code.
// ---------------------------------------------------------------------------
//
// MODE 1 (vvvv two-body density, first stage) reuses the tile loop for
// W_(ab),(cd) = sum_K T_(ab),K T'_(cd),K: both operand rows are consecutive
// (rows a_first.. of the left table, rows 0.. of the right one), m = (a, b)
// with b = m % vc, n = (c, d) with d = n % vd, and the element is stored at
// row (a - ga0) * nb + c, column xrow0 + b * vd + d of the region (no 1/2).
template <int BM, int BN, int MODE = 0>
__global__ __launch_bounds__(256) void assemble_f64_kernel(const P1Desc *__restrict__ descs,
                                                           const Tile *__restrict__ tiles, Queues Q,
                                                           int *__restrict__ cnt,
                                                           const SysPtrs *__restrict__ sp,
                                                           double *__restrict__ xbuf) {
  constexpr int BK = 16;
  // LDS tiles row-major like the operands ([row][k]) with a row stride of
  // BK + 1 doubles (34 banks): a thread's four consecutive k of one row go to
  // consecutive words, and the four threads of one k slot in a 16-lane group
  // (rows lr .. lr+3, k slots 0/4/8/12) land on 16 different bank pairs; a
  // fragment read (16 consecutive rows, one k) steps 34 words per lane, so
  // its 16 lanes cover the 32 banks once.  Both are free of bank conflicts.
  constexpr int LK = BK + 1;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int RA = BM / 64, RB = BN / 64;  // row slots per thread
  __shared__ double As[2][BM][LK];
  __shared__ double Bs[2][BN][LK];
  __shared__ int s_tile;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = tid >> 2, lk = (tid & 3) * 4;
  unsigned dead = 0;

  for (;;) {
    const int t = next_tile(cnt, Q, dead, &s_tile);
    if (t < 0) break;
    const Tile tl = tiles[t];
    const P1Desc D = descs[tl.desc];
    const double *__restrict__ op = sp[D.sys].opnd;
    const int m0 = tl.tm * BM, n0 = tl.tn * BN;
    const int K = D.K;

    // rows past M / N read a clamped row: they only reach results that are
    // never stored
    const CDCC_GLOBAL double *arow[RA];
    const CDCC_GLOBAL double *brow[RB];
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int m = min(m0 + lr + 64 * q, D.M - 1);
      arow[q] = as_global(op) + D.aoff + int64_t(m) * K + lk;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int nn = min(n0 + lr + 64 * q, D.N - 1);
      if constexpr (MODE == 1) {
        brow[q] = as_global(op) + D.boff + int64_t(nn) * K + lk;
      } else {
        const int dd = nn / D.nb, b = nn - dd * D.nb;
        brow[q] = as_global(op) + D.boff + (int64_t(b) * D.vd + dd) * K + lk;
      }
    }
    // 16-byte operand loads when every row starts on a 16-byte boundary
    const bool vec = ((D.aoff | D.boff | int64_t(K)) & 1) == 0 && (reinterpret_cast<uintptr_t>(op) & 15) == 0;

    d4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    double ra[RA][4], rb[RB][4];
    // a whole K block: no k mask; the right operand is negated from kneg on
    auto gload = [&](int k0) {
      if (vec) {
#pragma unroll
        for (int q = 0; q < RA; ++q) {
          const CDCC_GLOBAL d2 *p = reinterpret_cast<const CDCC_GLOBAL d2 *>(arow[q] + k0);
          const d2 u = p[0], v = p[1];
          ra[q][0] = u.x;
          ra[q][1] = u.y;
          ra[q][2] = v.x;
          ra[q][3] = v.y;
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const CDCC_GLOBAL d2 *p = reinterpret_cast<const CDCC_GLOBAL d2 *>(brow[q] + k0);
          const d2 u = p[0], v = p[1];
          rb[q][0] = u.x;
          rb[q][1] = u.y;
          rb[q][2] = v.x;
          rb[q][3] = v.y;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
#pragma unroll
          for (int q = 0; q < RA; ++q) ra[q][e] = arow[q][k0 + e];
#pragma unroll
          for (int q = 0; q < RB; ++q) rb[q][e] = brow[q][k0 + e];
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const double sg = k0 + lk + e >= D.kneg ? -1.0 : 1.0;
#pragma unroll
        for (int q = 0; q < RB; ++q) rb[q][e] *= sg;
      }
    };
    // the last, partial block: k past K reads a clamped address, zeroed by a select
    auto gload_tail = [&](int k0) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = k0 + lk + e;
        const bool kin = k < K;
        const int kc = (kin ? k : K - 1) - lk;
        const double sg = k >= D.kneg ? -1.0 : 1.0;
#pragma unroll
        for (int q = 0; q < RA; ++q) {
          const double x = arow[q][kc];
          ra[q][e] = kin ? x : 0.0;
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
          const double x = brow[q][kc];
          rb[q][e] = kin ? sg * x : 0.0;
        }
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int q = 0; q < RA; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) As[buf][lr + 64 * q][lk + e] = ra[q][e];
#pragma unroll
      for (int q = 0; q < RB; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) Bs[buf][lr + 64 * q][lk + e] = rb[q][e];
    };

    const int nfull = K / BK, nk = (K + BK - 1) / BK;
    if (nfull > 0) gload(0);
    else if (nk > 0) gload_tail(0);
    if (nk > 0) lstore(0);
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
        for (int i = 0; i < FM; ++i) fa[i] = As[cur][wm * WM + i * 16 + (lane & 15)][kr];
#pragma unroll
        for (int j = 0; j < FN; ++j) fb[j] = Bs[cur][wn * WN + j * 16 + (lane & 15)][kr];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], fb[j], acc[i][j], 0, 0, 0);
      }
      if (kn < nk) lstore(cur ^ 1);
      __syncthreads();
    }

    // epilogue: permuted store into the column group's X region.  The
    // quotients of a lane's rows (by vc) and columns (by nb or vd) are formed
    // once per row and per column, not once per element.
    int rq[FM][4], rrem[FM][4], cq[FN], crem[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * WM + i * 16 + (lane >> 4) + 4 * r;
        rq[i][r] = m / D.vc;
        rrem[i][r] = m - rq[i][r] * D.vc;
      }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int n = n0 + wn * WN + j * 16 + (lane & 15);
      const int dv = MODE == 1 ? D.vd : D.nb;
      cq[j] = n / dv;
      crem[j] = n - cq[j] * dv;
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * WM + i * 16 + (lane >> 4) + 4 * r;
          const int n = n0 + wn * WN + j * 16 + (lane & 15);
          if (m >= D.M || n >= D.N) continue;
          if constexpr (MODE == 1) {
            const int am = rq[i][r], b = rrem[i][r];
            const int c = cq[j], d = crem[j];
            const int64_t wrow = int64_t(D.a_first + am - D.ga0) * D.nb + c;
            xbuf[D.xoff + wrow * D.ldx + D.xrow0 + int64_t(b) * D.vd + d] = acc[i][j][r];
            continue;
          }
          const int a = D.a_first + rq[i][r], c = rrem[i][r];
          const int dd = cq[j], b = crem[j];
          if (D.tri && b > a) continue;
          const int64_t xcol = D.tri ? (int64_t(a) * (a + 1) / 2 - int64_t(D.ga0) * (D.ga0 + 1) / 2 + b)
                                     : (int64_t(a - D.ga0) * D.vb + b);
          const int64_t xrow = D.xrow0 + int64_t(c) * D.vd + dd;
          xbuf[D.xoff + xrow * D.ldx + xcol] = 0.5 * acc[i][j][r];
        }
  }
}

// Unpack one (S, A) pair of packed row m (i>=j) and group column n (a>=b)
// into R: (ij,ab) = S+A, (ij,ba) = (ji,ab) = S-A, (ji,ba) = S+A; and R/D.
__device__ __forceinline__ void unpack_store(const SysPtrs &S, const P2Group &g, int m, int n, double sv,
                                             double av, const int4 *__restrict__ ijtab,
                                             const int4 *__restrict__ vvtab) {
  const int4 ij = ijtab[g.ij_off + m];
  const int4 ab = vvtab[g.col_off + n];
  const bool oab = ab.x != ab.y, oij = ij.x != ij.y;
  // On a column a = b, W(-) is X_cd^aa - X_dc^aa = 0 identically (both are
  // sum_P B_ac^P B_ad^P).  The split-precision assemblies round the two
  // operand orders differently, so the exact zero is restored here; this
  // keeps R_ij^aa = R_ji^aa bitwise in every precision.
  if (!oab) av = 0.0;
  const double pp = sv + av, pm = sv - av;
  const int64_t ld = g.ldr;
  double *__restrict__ R = S.R + g.r_off;
  R[int64_t(ij.x) * ld + ab.x] = pp;
  if (oab) R[int64_t(ij.x) * ld + ab.y] = pm;
  if (oij) R[int64_t(ij.y) * ld + ab.x] = pm;
  if (oab && oij) R[int64_t(ij.y) * ld + ab.y] = pp;
  if (S.delta) {
    double *__restrict__ Dl = S.delta + g.r_off;
    const double den = (S.eps_occ[ij.z] + S.eps_occ[ij.w]) - (S.eps_vir[ab.z] + S.eps_vir[ab.w]);
    const double inv = 1.0 / den;
    Dl[int64_t(ij.x) * ld + ab.x] = pp * inv;
    if (oab) Dl[int64_t(ij.x) * ld + ab.y] = pm * inv;
    if (oij) Dl[int64_t(ij.y) * ld + ab.x] = pm * inv;
    if (oab && oij) Dl[int64_t(ij.y) * ld + ab.y] = pp * inv;
  }
}

// ---------------------------------------------------------------------------
// contract (FP64): S = tauhat(+) W(+), A = tauhat(-) W(-) over the K table of
// the group (entries: tauhat column, X rows of (c,d) and (d,c), -1 = absent).
// One workgroup of four waves per tile of 16*FM packed (ij) rows x 32 group
// columns.  The waves take interleaved K steps of four table entries (wave w:
// steps w, w+4, ...) and stream their operands from global memory straight
// into MFMA registers: tauhat is stored column-major (k-major), so a lane
// quarter reads 16 consecutive rows of one column; the X rows of (c,d) and
// (d,c) are summed and subtracted in registers.  A ring of NS stages keeps
// table entries 2*NS steps and data NS steps ahead; the K loop has no LDS
// traffic and no barrier.  The four partial sums are combined in LDS in the
// fixed order (w0 + w2) + (w1 + w3), so every element depends only on the
// group's K table and segment length, never on the tile shape.
// ---------------------------------------------------------------------------
constexpr int kCtBN = 32;                     // group columns per tile
constexpr int kCtMaxBM = 64;                  // rows per tile for FM = 4

// prefetch stages: fewer for the widest tile, whose accumulators take half
// of the 256 registers a wave has at two waves per SIMD
template <int FM>
struct CtStages {
  static constexpr int value = FM == 4 ? 2 : (FM == 3 ? 4 : (FM == 2 ? 6 : 8));
};

template <int FM>
__device__ __forceinline__ void contract_tile(const P2Group &g, const Tile &tl, const SysPtrs &S,
                                              const double *__restrict__ xbuf, const int4 *__restrict__ ktab,
                                              const int4 *__restrict__ ijtab, const int4 *__restrict__ vvtab,
                                              double *__restrict__ part, double (*red)[2 * kCtMaxBM * kCtBN]) {
  constexpr int FN = 2, BN = kCtBN, BM = 16 * FM, NS = CtStages<FM>::value;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int kq = lane >> 4, li = lane & 15;
  const int m0 = tl.tm * BM, n0 = tl.tn * BN;
  const int kbeg = tl.aux * g.kseg;
  const int klen = g.nsplit > 1 ? (g.ktab_len - kbeg < g.kseg ? g.ktab_len - kbeg : g.kseg) : g.ktab_len;
  const int ns = klen / 16;  // K steps of each wave (segments are multiples of 16 entries)
  const CDCC_GLOBAL int *gkt = as_global(reinterpret_cast<const int *>(ktab + g.ktab_off + kbeg));
  const CDCC_GLOBAL double *thp = as_global(S.tauhat) + g.th_off;  // [kcol][th_rs]
  const CDCC_GLOBAL double *thm = thp + int64_t(g.th_rs) * g.th_ld;
  const CDCC_GLOBAL double *gx = as_global(xbuf) + g.xoff;

  // rows and columns past the tile's edge read clamped addresses; they only
  // feed result rows / columns that are never stored, so need no mask
  int rowc[FM], colc[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int m = m0 + 16 * i + li;
    rowc[i] = m < g.n_ij ? m : g.n_ij - 1;
  }
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int n = n0 + 16 * j + li;
    colc[j] = n < g.ncols ? n : g.ncols - 1;
  }

  d4 accS[FM][FN], accA[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      accS[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      accA[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  if (ns > 0) {
    int kc[NS], r1[NS], r2[NS], fl[NS];
    double ap[NS][FM], am[NS][FM], x1[NS][FN], x2[NS][FN];
    // raw table entry of this lane for wave step s (index clamped into the
    // segment); the values are not touched here, so the loads stay in flight
    auto ktload = [&](int q, int s) {
      const int e0 = 4 * (4 * s + w) + kq;
      const int e = e0 < klen ? e0 : klen - 1;
      kc[q] = gkt[4 * e];
      r1[q] = gkt[4 * e + 1];
      r2[q] = gkt[4 * e + 2];
    };
    // operands of wave step s, whose entry is in slot q, from clamped
    // addresses; which of them are present is kept in fl[q] and applied
    // when they are used, so no instruction waits on these loads until then
    // (steps past the end load but count as absent)
    auto dload = [&](int q, int s) {
      // widest tile: an empty asm takes this stage's table entry here, so the
      // optimiser cannot start the next stage's address arithmetic early and
      // wait there for the youngest load in flight (every load of the ring)
      if constexpr (FM == 4) __asm__ volatile("" : "+v"(kc[q]), "+v"(r1[q]), "+v"(r2[q]));
      const bool in = s < ns;
      fl[q] = ((in && kc[q] >= 0) ? 1 : 0) | ((in && r1[q] >= 0) ? 2 : 0) | ((in && r2[q] >= 0) ? 4 : 0);
      const int64_t ko = int64_t(kc[q] >= 0 ? kc[q] : 0) * g.th_rs;
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ap[q][i] = thp[ko + rowc[i]];
        am[q][i] = thm[ko + rowc[i]];
      }
      const int64_t o1 = int64_t(r1[q] >= 0 ? r1[q] : 0) * g.ldx, o2 = int64_t(r2[q] >= 0 ? r2[q] : 0) * g.ldx;
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        x1[q][j] = gx[o1 + colc[j]];
        x2[q][j] = gx[o2 + colc[j]];
      }
    };
    auto mfma = [&](int q) {
      // an empty asm that takes and returns each loaded value: the wait for
      // these loads lands here, and no arithmetic on them is moved above it
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        __asm__ volatile("" : "+v"(ap[q][i]));
        __asm__ volatile("" : "+v"(am[q][i]));
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        __asm__ volatile("" : "+v"(x1[q][j]));
        __asm__ volatile("" : "+v"(x2[q][j]));
      }
      const bool ha = fl[q] & 1, h1 = fl[q] & 2, h2 = fl[q] & 4;
      double fa[FM], fb[FM], bp[FN], bmv[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        fa[i] = ha ? ap[q][i] : 0.0;
        fb[i] = ha ? am[q][i] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        const double v1 = h1 ? x1[q][j] : 0.0, v2 = h2 ? x2[q][j] : 0.0;
        bp[j] = v1 + v2;
        bmv[j] = v1 - v2;
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          accS[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[i], bp[j], accS[i][j], 0, 0, 0);
          accA[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fb[i], bmv[j], accA[i][j], 0, 0, 0);
        }
    };
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      ktload(q, q);
      fl[q] = 0;
#pragma unroll
      for (int i = 0; i < FM; ++i) ap[q][i] = am[q][i] = 0.0;
#pragma unroll
      for (int j = 0; j < FN; ++j) x1[q][j] = x2[q][j] = 0.0;
    }
    // stage q holds data of step s0 + q and the table entry of step
    // s0 + q + NS.  The first pass (s0 = -NS) only loads; the ring starts
    // from registers, not loads, so the compiler keeps the loads of a pass
    // in flight across the next one.  Steps past the end are zero.
    for (int s0 = -NS; s0 < ns; s0 += NS) {
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        if (s0 >= 0) mfma(q);
        dload(q, s0 + q + NS);
        ktload(q, s0 + q + 2 * NS);
        // compiler-only barrier: keeps the optimiser from turning the
        // loop-carried loaded values into loads at the top of the next pass
        // and the scheduler from hoisting a later stage's address
        // arithmetic (which waits for its table entry) above this stage
        __asm__ volatile("" ::: "memory");
      }
    }
  }

  // fixed-order combination of the four wave partials through LDS
  auto put = [&](double *dst) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = (16 * i + kq + 4 * r) * BN + 16 * j + li;
          dst[e] = accS[i][j][r];
          dst[BM * BN + e] = accA[i][j][r];
        }
  };
  auto add = [&](const double *src) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = (16 * i + kq + 4 * r) * BN + 16 * j + li;
          accS[i][j][r] += src[e];
          accA[i][j][r] += src[BM * BN + e];
        }
  };
  if (w >= 2) put(red[w - 2]);
  __syncthreads();
  if (w < 2) add(red[w]);
  __syncthreads();
  if (w == 1) put(red[0]);
  __syncthreads();
  if (w == 0) {
    add(red[0]);
    put(red[1]);
  }
  __syncthreads();

  const double *fin = red[1];
  if (g.nsplit > 1) {
    // this segment's S and A partials; the reduce kernel sums the segments
    // in order and unpacks
    double *__restrict__ pb = part + g.part_off + (int64_t(tl.tm * g.tiles_n + tl.tn) * g.nsplit + tl.aux) * (2 * BM * BN);
    for (int e = tid; e < 2 * BM * BN; e += 256) pb[e] = fin[e];
    return;
  }
  for (int e = tid; e < BM * BN; e += 256) {
    const int lm = e / BN, ln = e - lm * BN;
    const int m = m0 + lm, n = n0 + ln;
    if (m >= g.n_ij || n >= g.ncols) continue;
    unpack_store(S, g, m, n, fin[e], fin[BM * BN + e], ijtab, vvtab);
  }
}

__global__ __launch_bounds__(256, 2) void contract_f64_kernel(const P2Group *__restrict__ groups,
                                                              const Tile *__restrict__ tiles, Queues Q,
                                                              int *__restrict__ cnt,
                                                              const SysPtrs *__restrict__ sp,
                                                              const double *__restrict__ xbuf,
                                                              const int4 *__restrict__ ktab,
                                                              const int4 *__restrict__ ijtab,
                                                              const int4 *__restrict__ vvtab,
                                                              double *__restrict__ part) {
  __shared__ double red[2][2 * kCtMaxBM * kCtBN];
  __shared__ int s_tile;
  unsigned dead = 0;
  for (;;) {
    const int t = next_tile(cnt, Q, dead, &s_tile);
    if (t < 0) break;
    const Tile tl = tiles[t];
    const P2Group g = groups[tl.desc];
    const SysPtrs S = sp[g.sys];
    switch (g.fm) {
      case 1: contract_tile<1>(g, tl, S, xbuf, ktab, ijtab, vvtab, part, red); break;
      case 2: contract_tile<2>(g, tl, S, xbuf, ktab, ijtab, vvtab, part, red); break;
      case 3: contract_tile<3>(g, tl, S, xbuf, ktab, ijtab, vvtab, part, red); break;
      default: contract_tile<4>(g, tl, S, xbuf, ktab, ijtab, vvtab, part, red); break;
    }
  }
}

// ---------------------------------------------------------------------------
// reduce (split K): one workgroup per contraction tile; S and A summed over
// the K segments in segment order, then the same unpack as above.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void reduce_unpack_kernel(const P2Group *__restrict__ groups,
                                                            const Tile *__restrict__ jobs,
                                                            const SysPtrs *__restrict__ sp,
                                                            const double *__restrict__ part,
                                                            const int4 *__restrict__ ijtab,
                                                            const int4 *__restrict__ vvtab) {
  const Tile tl = jobs[blockIdx.x];
  const P2Group g = groups[tl.desc];
  const SysPtrs S = sp[g.sys];
  const int BM = 16 * g.fm, BN = kCtBN;
  const double *__restrict__ pb =
      part + g.part_off + int64_t(tl.tm * g.tiles_n + tl.tn) * g.nsplit * (2 * BM * BN);
  for (int e = threadIdx.x; e < BM * BN; e += 256) {
    const int lm = e / BN, ln = e - lm * BN;
    const int m = tl.tm * BM + lm, n = tl.tn * BN + ln;
    if (m >= g.n_ij || n >= g.ncols) continue;
    double sv = 0.0, av = 0.0;
    for (int k = 0; k < g.nsplit; ++k) {
      sv += pb[int64_t(k) * (2 * BM * BN) + e];
      av += pb[int64_t(k) * (2 * BM * BN) + BM * BN + e];
    }
    unpack_store(S, g, m, n, sv, av, ijtab, vvtab);
  }
}
// ---------------------------------------------------------------------------
// pair energies: one workgroup per amplitude row (i,j); fixed-order tree.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(512) void energy_kernel(const EnergyJob *__restrict__ jobs,
                                                     const SysPtrs *__restrict__ sp,
                                                     const int *__restrict__ vvfull) {
  constexpr int NT = 512, U = 4;
  __shared__ double red[NT];
  const EnergyJob J = jobs[blockIdx.x];
  const SysPtrs S = sp[J.sys];
  if (!S.epair) return;
  const CDCC_GLOBAL double *xr = as_global(S.eamp) + J.r_off + int64_t(J.row) * J.ldr;
  const CDCC_GLOBAL double *rr = as_global(S.R) + J.r_off + int64_t(J.row) * J.ldr;
  const CDCC_GLOBAL int *tc = as_global(vvfull) + J.vvfull_off;
  // U columns per thread per pass: all loads of a pass are issued before the
  // (in-order) accumulation
  double acc = 0.0;
  for (int c0 = threadIdx.x; c0 < J.ncol; c0 += NT * U) {
    double x[U], xt[U], r[U];
    int t[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * NT;
      const int cc = c < J.ncol ? c : J.ncol - 1;
      t[u] = tc[cc];
      x[u] = xr[cc];
      r[u] = rr[cc];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xt[u] = xr[t[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (c0 + u * NT < J.ncol) acc += (2.0 * x[u] - xt[u]) * r[u];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) S.epair[int64_t(J.I) * J.nocc_tot + J.J] = red[0];
}

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
hipError_t launch_fill_int(int *p, int n, int v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_int_kernel<<<(n + 255) / 256, 256, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_pack(const PackJob *jobs, const int2 *rows, int nrows, const SysPtrs *sp, const int4 *ijtab,
                       const int4 *vvtab, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  pack_kernel<<<nrows, 256, 0, s>>>(jobs, rows, sp, ijtab, vvtab);
  return hipGetLastError();
}

hipError_t launch_dress(const DressJob *jobs, const int2 *rows, int nrows, const SysPtrs *sp, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  dress_kernel<<<nrows, 256, 0, s>>>(jobs, rows, sp);
  return hipGetLastError();
}

hipError_t launch_assemble_f64(int cls, int grid, const P1Desc *descs, const Tile *tiles, const Queues &Q,
                               int *cnt, const SysPtrs *sp, double *xbuf, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  switch (cls) {
    case 0: assemble_f64_kernel<64, 64><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf); break;
    case 1: assemble_f64_kernel<128, 64><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf); break;
    default: assemble_f64_kernel<128, 128><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf); break;
  }
  return hipGetLastError();
}

// vvvv density, first stage (W = T T'^T with the density store): 128 x 64 tiles
hipError_t launch_assemble_density(int grid, const P1Desc *descs, const Tile *tiles, const Queues &Q, int *cnt,
                                   const SysPtrs *sp, double *xbuf, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  assemble_f64_kernel<128, 64, 1><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf);
  return hipGetLastError();
}

int occupancy_density_w() {
  int n = 0;
  const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_f64_kernel<128, 64, 1>, 256, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_contract_f64(int grid, const P2Group *groups, const Tile *tiles, const Queues &Q, int *cnt,
                               const SysPtrs *sp, const double *xbuf, const int4 *ktab, const int4 *ijtab,
                               const int4 *vvtab, double *part, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  contract_f64_kernel<<<grid, 256, 0, s>>>(groups, tiles, Q, cnt, sp, xbuf, ktab, ijtab, vvtab, part);
  return hipGetLastError();
}

hipError_t launch_reduce_unpack(int njobs, const P2Group *groups, const Tile *jobs, const SysPtrs *sp,
                                const double *part, const int4 *ijtab, const int4 *vvtab, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  reduce_unpack_kernel<<<njobs, 256, 0, s>>>(groups, jobs, sp, part, ijtab, vvtab);
  return hipGetLastError();
}

// Resident workgroups per CU (which: 0 = assemble, 1 = contract).
int occupancy_f64(int which, int cls) {
  int n = 0;
  hipError_t e;
  if (which == 0) {
    if (cls == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_f64_kernel<64, 64>, 256, 0);
    else if (cls == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_f64_kernel<128, 64>, 256, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_f64_kernel<128, 128>, 256, 0);
  } else {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, contract_f64_kernel, 256, 0);
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_energy(const EnergyJob *jobs, int njobs, const SysPtrs *sp, const int *vvfull, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  energy_kernel<<<njobs, 512, 0, s>>>(jobs, sp, vvfull);
  return hipGetLastError();
}

}  // namespace cdcc
