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

typedef double d4 __attribute__((ext_vector_type(4)));

// MFMA f64 16x16x4 lane mapping (gfx950): A[i][k] in lane i + 16k,
// B[k][j] in lane j + 16k, result register r of lane l is D[l/16 + 4r][l%16].

__global__ void fill_int_kernel(int *p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// pack: one workgroup per packed row (i>=j) of one (system, G).
//   tauhat(+)_ij^cd = X_ij^cd + X_ij^dc   (c>d),   X_ij^cc   (c=d)
//   tauhat(-)_ij^cd = X_ij^cd - X_ij^dc   (c>d),   0         (c=d or i=j)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pack_kernel(const PackJob *__restrict__ jobs,
                                                   const int2 *__restrict__ rows,
                                                   const SysPtrs *__restrict__ sp,
                                                   const int4 *__restrict__ ijtab,
                                                   const int4 *__restrict__ vvtab) {
  const int2 jr = rows[blockIdx.x];
  const PackJob J = jobs[jr.x];
  const int r = jr.y;
  const SysPtrs S = sp[J.sys];
  const int4 ij = ijtab[J.ij_off + r];
  const bool diag_ij = ij.x == ij.y;
  const double *__restrict__ xr = S.X + J.x_off + int64_t(ij.x) * J.ldx;
  double *__restrict__ tp = S.tauhat + J.th_off + int64_t(r) * J.ncol;
  double *__restrict__ tm = tp + int64_t(J.nrow) * J.ncol;
  for (int k = threadIdx.x; k < J.ncol; k += blockDim.x) {
    const int4 cd = vvtab[J.vv_off + k];
    const double x1 = xr[cd.x];
    const double x2 = xr[cd.y];
    const bool dcd = cd.x == cd.y;
    tp[k] = dcd ? x1 : x1 + x2;
    tm[k] = (dcd || diag_ij) ? 0.0 : x1 - x2;
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
// wave (BM/2) x (BN/2) as 16x16 MFMA f64 blocks.  LDS holds [k][row] (padded
// by 2 doubles, double-buffered, one barrier per K step).  Out-of-range rows
// and K are read from a clamped address and zeroed by a select, so the loads
// are straight-line code.
// ---------------------------------------------------------------------------
template <int BM, int BN>
__global__ __launch_bounds__(256) void assemble_f64_kernel(const P1Desc *__restrict__ descs,
                                                           const Tile *__restrict__ tiles, Queues Q,
                                                           int *__restrict__ cnt,
                                                           const SysPtrs *__restrict__ sp,
                                                           double *__restrict__ xbuf) {
  constexpr int BK = 16;
  constexpr int LA = BM + 2, LB = BN + 2;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int RA = BM / 64, RB = BN / 64;  // row slots per thread
  __shared__ double As[2][BK][LA];
  __shared__ double Bs[2][BK][LB];
  __shared__ int s_tile;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int lr = tid >> 2, lk = (tid & 3) * 4;
  int tries = 0;

  for (;;) {
    const int t = next_tile(cnt, Q, tries, &s_tile);
    if (t < 0) break;
    const Tile tl = tiles[t];
    const P1Desc D = descs[tl.desc];
    const double *__restrict__ op = sp[D.sys].opnd;
    const int m0 = tl.tm * BM, n0 = tl.tn * BN;
    const int K = D.K;

    const CDCC_GLOBAL double *arow[RA];
    const CDCC_GLOBAL double *brow[RB];
    double am[RA], bmk[RB];  // 1 for a real row, 0 for a padding row
#pragma unroll
    for (int q = 0; q < RA; ++q) {
      const int m = m0 + lr + 64 * q;
      am[q] = m < D.M ? 1.0 : 0.0;
      arow[q] = as_global(op) + D.aoff + int64_t(m < D.M ? m : D.M - 1) * K;
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const int n = n0 + lr + 64 * q;
      bmk[q] = n < D.N ? 1.0 : 0.0;
      const int nn = n < D.N ? n : D.N - 1;
      const int dd = nn / D.nb, b = nn - dd * D.nb;
      brow[q] = as_global(op) + D.boff + (int64_t(b) * D.vd + dd) * K;
    }

    d4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

    // loads are unconditional (clamped index) and masked by a multiply, so
    // the K loop is one basic block
    double ra[RA][4], rb[RB][4];
    auto gload = [&](int k0) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int k = k0 + lk + e;
        const bool kin = k < K;
        const int kc = kin ? k : K - 1;
        const double ka = kin ? 1.0 : 0.0;
        const double kb = kin ? (k >= D.kneg ? -1.0 : 1.0) : 0.0;
#pragma unroll
        for (int q = 0; q < RA; ++q) ra[q][e] = arow[q][kc] * (am[q] * ka);
#pragma unroll
        for (int q = 0; q < RB; ++q) rb[q][e] = brow[q][kc] * (bmk[q] * kb);
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int q = 0; q < RA; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) As[buf][lk + e][lr + 64 * q] = ra[q][e];
#pragma unroll
      for (int q = 0; q < RB; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) Bs[buf][lk + e][lr + 64 * q] = rb[q][e];
    };

    const int nk = (K + BK - 1) / BK;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int kb = 0; kb < nk; ++kb) {
      const int cur = kb & 1;
      // unconditional prefetch (clamped, zeroed past K): no branch, so the
      // wait for these loads lands after the MFMAs below
      gload((kb + 1) * BK);
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
      lstore(cur ^ 1);
      __syncthreads();
    }

    // epilogue: permuted store into the column group's X region
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm * WM + i * 16 + (lane >> 4) + 4 * r;
          const int n = n0 + wn * WN + j * 16 + (lane & 15);
          if (m >= D.M || n >= D.N) continue;
          const int am = m / D.vc, c = m - am * D.vc;
          const int a = D.a_first + am;
          const int dd = n / D.nb, b = n - dd * D.nb;
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
  const double pp = sv + av, pm = sv - av;
  const int64_t ld = g.ldr;
  const bool oab = ab.x != ab.y, oij = ij.x != ij.y;
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
// Tile BM x BN of (packed ij) x (group columns); 2x2 waves; both products
// share the staged X rows; double-buffered LDS, one barrier per K step.
// Epilogue writes R (and R/D) at the four permutations (ij,ab),
// (ij,ba) = S-A, (ji,ab) = S-A, (ji,ba) = S+A.
// ---------------------------------------------------------------------------
template <int BM, int BN, int NT, bool PARTIAL>
__global__ __launch_bounds__(NT) void contract_f64_kernel(const P2Group *__restrict__ groups,
                                                           const Tile *__restrict__ tiles, Queues Q,
                                                           int *__restrict__ cnt,
                                                           const SysPtrs *__restrict__ sp,
                                                           const double *__restrict__ xbuf,
                                                           const int4 *__restrict__ ktab,
                                                           const int4 *__restrict__ ijtab,
                                                           const int4 *__restrict__ vvtab,
                                                           double *__restrict__ part) {
  constexpr int BK = 16;
  constexpr int NW = NT / 64;                // waves: 2 along M, NW/2 along N
  constexpr int WM = BM / 2, WN = BN / (NW / 2);
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int EPT = BM * BK / NT;          // A elements per thread (one row, EPT consecutive k)
  constexpr int TPR = BK / EPT;              // threads per A row
  constexpr int CB = BN * BK / NT;           // B columns per thread (one k row)
  constexpr int TPK = BN / CB;               // threads per B k row
  constexpr int LA = BM + 2, LB = BN + 2;
  static_assert(EPT >= 1 && BK % EPT == 0 && CB >= 1 && FN >= 1, "staging");
  __shared__ double Ap[2][BK][LA], Am[2][BK][LA];
  __shared__ double Bp[2][BK][LB], Bm[2][BK][LB];
  __shared__ int s_tile;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int lr = tid / TPR, lk = (tid % TPR) * EPT;  // A staging
  const int bk = tid / TPK, bc = (tid % TPK) * CB;   // B staging
  int tries = 0;

  for (;;) {
    const int t = next_tile(cnt, Q, tries, &s_tile);
    if (t < 0) break;
    const Tile tl = tiles[t];
    const P2Group g = groups[tl.desc];
    const SysPtrs S = sp[g.sys];
    const int m0 = tl.tm * BM, n0 = tl.tn * BN;
    const CDCC_GLOBAL double *gthp = as_global(S.tauhat) + g.th_off;
    const CDCC_GLOBAL double *gthm = gthp + int64_t(g.n_ij) * g.th_ld;
    const CDCC_GLOBAL double *gxr = as_global(xbuf) + g.xoff;
    // K segment of this tile (the whole table unless the group is split)
    const int kbeg = tl.aux * g.kseg;
    const int klen = (g.nsplit > 1 ? (g.ktab_len - kbeg < g.kseg ? g.ktab_len - kbeg : g.kseg) : g.ktab_len);
    const CDCC_GLOBAL int *gkt = as_global(reinterpret_cast<const int *>(ktab + g.ktab_off + kbeg));  // int4 entries

    d4 accS[FM][FN], accA[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        accS[i][j] = d4{0.0, 0.0, 0.0, 0.0};
        accA[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      }

    const int r = m0 + lr;
    const int64_t arow = int64_t(r < g.n_ij ? r : g.n_ij - 1) * g.th_ld;
    const double rm = r < g.n_ij ? 1.0 : 0.0;
    double rap[EPT], ram[EPT], rbp[CB], rbm[CB];
    // K-table entries are fetched one stage ahead of the data they index
    int kcA[EPT], r1B, r2B;
    auto kload = [&](int k0) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) kcA[e] = gkt[4 * (k0 + lk + e)];
      r1B = gkt[4 * (k0 + bk) + 1];
      r2B = gkt[4 * (k0 + bk) + 2];
    };
    // branch-free staging: clamped indices, masked by a multiply
    auto gload = [&]() {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int kc = kcA[e];
        const double mk = kc >= 0 ? rm : 0.0;
        const int64_t off = arow + (kc >= 0 ? kc : 0);
        rap[e] = gthp[off] * mk;
        ram[e] = gthm[off] * mk;
      }
      const double m1 = r1B >= 0 ? 1.0 : 0.0, m2 = r2B >= 0 ? 1.0 : 0.0;
      const int64_t o1 = int64_t(r1B >= 0 ? r1B : 0) * g.ldx, o2 = int64_t(r2B >= 0 ? r2B : 0) * g.ldx;
#pragma unroll
      for (int e = 0; e < CB; ++e) {
        const int n = n0 + bc + e;
        const int nc = n < g.ncols ? n : g.ncols - 1;
        const double nm = n < g.ncols ? 1.0 : 0.0;
        const double x1 = gxr[o1 + nc] * (m1 * nm);
        const double x2 = gxr[o2 + nc] * (m2 * nm);
        rbp[e] = x1 + x2;
        rbm[e] = x1 - x2;
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        Ap[buf][lk + e][lr] = rap[e];
        Am[buf][lk + e][lr] = ram[e];
      }
#pragma unroll
      for (int e = 0; e < CB; ++e) {
        Bp[buf][bk][bc + e] = rbp[e];
        Bm[buf][bk][bc + e] = rbm[e];
      }
    };

    const int nk = klen / BK;
    if (nk > 0) {
      kload(0);
      gload();
      lstore(0);
      kload((nk > 1 ? 1 : 0) * BK);
    }
    __syncthreads();
    for (int kb = 0; kb < nk; ++kb) {
      const int cur = kb & 1;
      gload();                                       // stage kb+1 (redundant on the last step)
      kload((kb + 2 < nk ? kb + 2 : nk - 1) * BK);   // table entries of stage kb+2
#pragma unroll
      for (int ks = 0; ks < BK / 4; ++ks) {
        const int kr = ks * 4 + (lane >> 4);
        double fap[FM], fam[FM], fbp[FN], fbm[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          fap[i] = Ap[cur][kr][wm * WM + i * 16 + (lane & 15)];
          fam[i] = Am[cur][kr][wm * WM + i * 16 + (lane & 15)];
        }
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          fbp[j] = Bp[cur][kr][wn * WN + j * 16 + (lane & 15)];
          fbm[j] = Bm[cur][kr][wn * WN + j * 16 + (lane & 15)];
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            accS[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fap[i], fbp[j], accS[i][j], 0, 0, 0);
            accA[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fam[i], fbm[j], accA[i][j], 0, 0, 0);
          }
      }
      lstore(cur ^ 1);
      __syncthreads();
    }

    if (PARTIAL || g.nsplit > 1) {
      // store this segment's S and A partials; the reduce kernel sums the
      // segments in order and unpacks (PARTIAL: always, to keep the unpack
      // epilogue out of this kernel's register budget)
      double *__restrict__ pb =
          part + g.part_off + (int64_t(tl.tm * g.tiles_n + tl.tn) * g.nsplit + tl.aux) * (2 * BM * BN);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int lm = wm * WM + i * 16 + (lane >> 4) + 4 * rr;
            const int ln = wn * WN + j * 16 + (lane & 15);
            pb[lm * BN + ln] = accS[i][j][rr];
            pb[BM * BN + lm * BN + ln] = accA[i][j][rr];
          }
      continue;
    }
    if constexpr (!PARTIAL) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int m = m0 + wm * WM + i * 16 + (lane >> 4) + 4 * rr;
            const int n = n0 + wn * WN + j * 16 + (lane & 15);
            if (m >= g.n_ij || n >= g.ncols) continue;
            unpack_store(S, g, m, n, accS[i][j][rr], accA[i][j][rr], ijtab, vvtab);
          }
    }
  }
}

// ---------------------------------------------------------------------------
// reduce (split K): one workgroup per contraction tile; S and A summed over
// the K segments in segment order, then the same unpack as above.
// ---------------------------------------------------------------------------
template <int BM, int BN>
__global__ __launch_bounds__(256) void reduce_unpack_kernel(const P2Group *__restrict__ groups,
                                                            const Tile *__restrict__ jobs,
                                                            const SysPtrs *__restrict__ sp,
                                                            const double *__restrict__ part,
                                                            const int4 *__restrict__ ijtab,
                                                            const int4 *__restrict__ vvtab) {
  const Tile tl = jobs[blockIdx.x];
  const P2Group g = groups[tl.desc];
  const SysPtrs S = sp[g.sys];
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
__global__ __launch_bounds__(256) void energy_kernel(const EnergyJob *__restrict__ jobs,
                                                     const SysPtrs *__restrict__ sp,
                                                     const int *__restrict__ vvfull) {
  __shared__ double red[256];
  const EnergyJob J = jobs[blockIdx.x];
  const SysPtrs S = sp[J.sys];
  if (!S.epair) return;
  const double *__restrict__ xr = S.X + J.r_off + int64_t(J.row) * J.ldr;
  const double *__restrict__ rr = S.R + J.r_off + int64_t(J.row) * J.ldr;
  const int *__restrict__ tc = vvfull + J.vvfull_off;
  double acc = 0.0;
  for (int c = threadIdx.x; c < J.ncol; c += 256) acc += (2.0 * xr[c] - xr[tc[c]]) * rr[c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
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

// Contraction tile classes: 0 = 32 x 64, 1 = 64 x 64 (LDS kernel, unpack in
// the epilogue unless split), 2 = 128 x 64 (always through the partial buffer).
hipError_t launch_contract_f64(int cls, int grid, const P2Group *groups, const Tile *tiles, const Queues &Q, int *cnt,
                               const SysPtrs *sp, const double *xbuf, const int4 *ktab, const int4 *ijtab,
                               const int4 *vvtab, double *part, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  switch (cls) {
    case 0:
      contract_f64_kernel<32, 64, 256, false><<<grid, 256, 0, s>>>(groups, tiles, Q, cnt, sp, xbuf, ktab, ijtab, vvtab, part);
      break;
    case 1:
      contract_f64_kernel<64, 64, 256, false><<<grid, 256, 0, s>>>(groups, tiles, Q, cnt, sp, xbuf, ktab, ijtab, vvtab, part);
      break;
    default:
      contract_f64_kernel<128, 64, 256, true><<<grid, 256, 0, s>>>(groups, tiles, Q, cnt, sp, xbuf, ktab, ijtab, vvtab, part);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_reduce_unpack(int cls, int njobs, const P2Group *groups, const Tile *jobs, const SysPtrs *sp,
                                const double *part, const int4 *ijtab, const int4 *vvtab, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  switch (cls) {
    case 0: reduce_unpack_kernel<32, 64><<<njobs, 256, 0, s>>>(groups, jobs, sp, part, ijtab, vvtab); break;
    case 1: reduce_unpack_kernel<64, 64><<<njobs, 256, 0, s>>>(groups, jobs, sp, part, ijtab, vvtab); break;
    default: reduce_unpack_kernel<128, 64><<<njobs, 256, 0, s>>>(groups, jobs, sp, part, ijtab, vvtab); break;
  }
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
    if (cls == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, contract_f64_kernel<32, 64, 256, false>, 256, 0);
    else if (cls == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, contract_f64_kernel<64, 64, 256, false>, 256, 0);
    else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, contract_f64_kernel<128, 64, 256, true>, 256, 0);
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_energy(const EnergyJob *jobs, int njobs, const SysPtrs *sp, const int *vvfull, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  energy_kernel<<<njobs, 256, 0, s>>>(jobs, sp, vvfull);
  return hipGetLastError();
}

}  // namespace cdcc
