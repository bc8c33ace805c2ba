// Device-visible descriptors shared by the host planner and the HIP kernels.
// All structs are plain data, 8-byte aligned, copied to device memory once per
// plan (tables) or once per call (pointers).
#pragma once
#include <stdint.h>

namespace cdcc {

// Per-system device pointers of one call.
struct SysPtrs {
  const double *opnd;    // operand of the (ac|bd) assembly: B (T2) or the dressed stack U (Lambda)
  const double *X;       // tau or lambda, full DPD storage
  double *R;             // result
  double *delta;         // optional R / D
  const double *eps_occ; // optional
  const double *eps_vir; // optional
  double *epair;         // optional pair energies
  double *tauhat;        // workspace: packed +/- amplitudes of this system
  const double *B;       // raw Cholesky vectors (Lambda dressing input)
  const double *Bvo;     // optional vo block (Lambda)
  const double *t1;      // optional singles (Lambda)
  unsigned char *slices; // workspace: sliced assembly operand (split paths: BF16 or 8-bit digits)
  double *rowscale;      // workspace: per-row power-of-two scales of the operand (mixed path)
  const double *eamp;    // amplitudes T of the pair energies (energy_amps, else X)
};

// Packing of X into the +/- halves for one (system, pair irrep G).
struct PackJob {
  int32_t sys, nrow, ncol, ldx;   // nrow = n_oo_pk(G), ncol = n_vv_pk(G), ldx = n_vv(G)
  int32_t ij_off, vv_off;
  int32_t ldt;                    // tauhat column stride (k-major halves, >= nrow)
  int32_t pad1;
  int64_t x_off;                  // amp_off[G]
  int64_t th_off;                 // element offset of tauhat(+) in SysPtrs::tauhat; (-) follows
};

// One GEMM of the (ac|bd) assembly: rows (a,c) for a in [a_first, a_first+na),
// c in Gc; columns (d,b) with b fastest; K = Cholesky index (x2 for Lambda).
struct P1Desc {
  int32_t sys, M, N, K;
  int32_t kneg;        // K index from which the right operand is negated (Lambda stack)
  int32_t vc, vd, vb;  // extents of c, d and b
  int32_t nb;          // number of b values covered (vb, or a_last+1 when Ga == Gb)
  int32_t a_first;     // first a of the rows
  int32_t ga0;         // first a of the owning column group (column numbering)
  int32_t tri;         // Ga == Gb: only b <= a is stored
  int32_t ldx, xrow0;  // X region row length; first region row of this Gc block
  int32_t Kp;          // split paths: padded K of a sliced row (multiple of the K block)
  int32_t kneg_blk;    // split paths: first K block (16 wide BF16, 32 wide 8-bit) of the subtracted half
  int64_t aoff;        // element offset of operand row (a_first, c=0)
  int64_t boff;        // element offset of operand row (b=0, d=0) of block (GP, Gb)
  int64_t xoff;        // element offset of the group's X region in the batch buffer
  int64_t a_soff;      // split paths: byte offset of sliced row (a_first, c=0)
  int64_t b_soff;      // split paths: byte offset of sliced row (0, 0) of block (GP, Gb)
  int64_t a_scoff;     // mixed path: row-scale index of row (a_first, c=0)
  int64_t b_scoff;     // mixed path: row-scale index of row (0, 0) of block (GP, Gb)
};

// One column group: the (a,b) pairs with a in [a0, a0+na) of sub-block (Ga, Gb)
// of pair irrep G, numbered like the packed a>=b list.
struct P2Group {
  int32_t sys, G, n_ij, ncols;
  int32_t ldx, ktab_len, ktab_off, ij_off;
  int32_t col_off;     // offset into the vv-pair table for column 0 of the group
  int32_t ldr;         // n_vv(G): R row length
  int32_t th_ld;       // n_vv_pk(G): tauhat row length
  int32_t kseg;        // K-table entries per split-K segment (multiple of 16)
  int32_t nsplit;      // number of K segments (1: the tile writes R itself)
  int32_t tiles_n;     // column tiles of the group (partial-block numbering)
  int32_t fm;          // 16-row MFMA fragments per contraction tile (tile rows = 16 fm)
  int32_t th_rs;       // tauhat column stride (k-major: element (ij, k) at k * th_rs + ij)
  int64_t xoff;        // X region in the batch buffer
  int64_t th_off;      // tauhat(+) offset; (-) at th_off + th_rs * th_ld
  int64_t r_off;       // amp_off[G]
  int64_t part_off;    // first partial block of the group in the split-K buffer
};

// Per-row data of the pair-energy reduction.
struct EnergyJob {
  int32_t sys, ncol, ldr, vvfull_off;
  int32_t row, I, J, nocc_tot;
  int64_t r_off;
};

struct Tile {
  int32_t desc, tm, tn, aux;   // aux: K segment of a split contraction tile
};

// Per-XCD tile queues of one launch: queue x holds tiles [qb[x], qb[x+1]) of
// the launch's tile list.  Workgroup w runs on XCD w % 8, drains queue w % 8
// first and then steals from the others, so every workgroup ends.
struct Queues {
  int32_t qb[9];
};

// Queue counters of one launch sit kQueueStride ints (256 bytes) apart, each
// in a cache line of its own, so claims on different queues do not serialise
// on one line.
constexpr int kQueueStride = 64;


// Lambda dressing of one (system, GP, Ga) block.
struct DressJob {
  int32_t sys, va, ve, np;   // rows a, columns e (Ge = Ga ^ GP), Cholesky count
  int32_t om, pad0, pad1, pad2;  // occupied count of irrep Ge
  int64_t u_off;             // U block (a, e, 2np)
  int64_t b_off;             // B block (GP, Ge): [e][a][P]
  int64_t bvo_off;           // Bvo block (GP, Ga): [a][m][P]
  int64_t t1_off;            // t1 block Ge: [m][e]
};

// Slicing of one operand block (split paths): rows of length K = halves * np
// (the Lambda stack has two halves), written as Kp = halves * roundup(np, kb)
// padded K, four slices per element: BF16 (kb = 16, 8 bytes per element) or
// 8-bit digits (kb = 32, 4 bytes per element).
struct SliceJob {
  int32_t sys, rows, np, halves;
  int32_t Kp;
  int32_t dress;       // 1: rows of the Lambda stack built here from B, L and t1 (no U)
  int32_t ve, om;      // dress: rows are (a, e), e fastest; om = occupied count of irrep Ge
  int64_t src_off;     // element offset of row 0 in the operand (dress == 0)
  int64_t dst_off;     // byte offset of row 0 in the slice buffer
  int64_t scale_off;   // row-scale index of row 0
  int64_t b_off;       // dress: B block (GP, Ge), [e][a][P]
  int64_t bvo_off;     // dress: L block (GP, Ga), [a][m][P]
  int64_t t1_off;      // dress: t1 block Ge, [m][e]
};

// vvvv two-body density: per-system pointers.
struct DensPtrs {
  const double *X;     // tau~ amplitudes (amplitude layout)
  const double *Y;     // lambda amplitudes (amplitude layout)
  const double *L;     // transformed Cholesky vectors (Cholesky layout)
  double *G;           // result G^P_ac (Cholesky layout)
  double *T;           // workspace: per pair irrep, rows (ab) of [Y | X], then rows (cd) of
                       // [2X^cd - X^dc | 2Y^cd - Y^dc] (the spin-adapted exchange partner)
};

// Transposition of one pair-irrep amplitude block into the T tables.
struct DensPackJob {
  int32_t sys, nrow, ncol;         // nrow = n_oo(G) (K half), ncol = n_vv(G) (pair rows)
  int32_t sw_off;                  // column swap table entries [sw_off, sw_off + ncol): column of (d,c)
  int64_t x_off;                   // amp_off[G]
  int64_t tw_off;                  // element offset of row 0 of [Y | X] in T; [X | Y] follows
};

// One plain GEMM of the second stage: C = alpha A B, A rows K-contiguous
// (lda, a multiple of 4), B row-major [K][N] (ldb), C row-major (ldc).
// K is cut into segments of kGemmKSeg (the last one shorter); with more than
// one segment every segment writes its BM x BN partial tile and a reduction
// sums them in segment order, so the result depends on K only, not on the
// batch the GEMM runs in.
constexpr int kGemmKSeg = 2048;
constexpr int kGemmBM = 128, kGemmBN = 64;
struct GemmDesc {
  int32_t sys, M, N, K;
  int32_t lda, ldb, ldc, nseg;
  int32_t tiles_n, pad0;
  int64_t aoff;        // into the batch buffer
  int64_t boff;        // into DensPtrs::L
  int64_t coff;        // into DensPtrs::G
  int64_t poff;        // into the partial-tile buffer (nseg > 1): [tm][tn][seg][BM * BN]
  double alpha;
};

// Partial symmetric-antisymmetric contraction M_bi^dc = sum_mn lam_bi^mn
// tau_mn^dc: per-system pointers.
struct PmPtrs {
  const double *lam;   // lambda_bi^mn (vo layout)
  const double *tau;   // tau~_mn^dc (amplitude layout, pair symmetric)
  double *M;           // result (vo layout)
  double *ws;          // workspace: packed lam+/lam- and tau+/tau- of this system
};

// One (system, pair irrep G) block.  K = the m >= n pairs of G (kp table
// entries [kp_off, kp_off + nk): oo-column indices of (m,n) and (n,m)),
// padded with zeros to ldk (a multiple of 16).  Columns = squares of 8 d x 8
// c (square table entries [sq_off, sq_off + nsq)), 64 columns each.
struct PmDesc {
  int32_t sys, nrow, nk, ldk;     // nrow = n_vo(G)
  int32_t nsq, kp_off, sq_off, pad0;
  int64_t lam_off;                // block of lambda (n_vo x n_oo)
  int64_t tau_off;                // block of tau (n_oo x n_vv)
  int64_t m_off;                  // block of M (n_vo x n_vv)
  int64_t n_oo, n_vv;             // row strides of lambda and of tau / M
  int64_t lp_off;                 // ws: lam+ [nrow][ldk], lam- follows
  int64_t tp_off;                 // ws: tau+ [ldk][nsq * 64], tau- follows
};

// A square of the d >= c column pairs: d in [d0, d0 + nd) of irrep Gd, c in
// [c0, c0 + nc) of irrep Gc (Gd > Gc, or Gd == Gc and the d block at or
// after the c block).  Column of (d,c) in the amplitude layout:
// base_dc + dd * ld_dc + cc; column of (c,d): base_cd + cc * ld_cd + dd
// (dd, cc local to the square).  diag: the square sits on the d = c block
// diagonal and holds both orders, so only (d,c) is written.
struct PmSquare {
  int32_t base_dc, base_cd, ld_dc, ld_cd;
  int32_t nd, nc, diag, pad0;
};

// Work of the +/- packing kernels: one chunk of 256 elements of one block.
struct PmChunk {
  int32_t desc, chunk;
};

// Two-step Cholesky decomposition.  Qualified pairs of one macro iteration:
// irrep, row (pair index in the irrep) and column slot in the irrep's
// residual block.
constexpr int kCdQmaxCap = 2048;
struct CdQ {
  int32_t g, r, slot, pad0;
};

// Per-irrep device buffers of the first step.
struct CdPtrs {
  double *D[8];          // diagonals (n)
  uint8_t *inP[8];       // membership of P (n)
  double *L1[8];         // vectors so far, [r][p], ld n (capacity n vectors)
  double *M[8];          // residual columns of the qualified pairs, [r][slot], ld qcap
  int32_t *piv[8];       // pivots in the order chosen (capacity n)
  int32_t *qpos[8];      // row -> its slot in the irrep's part of the qualified list, or -1
  int64_t n[8];
  int32_t qcap[8];
};

// Device-side state of the micro iterations.  The irreps run their micro
// iterations side by side (one step of every irrep per launch): a step of
// irrep g changes only the diagonals of irrep g, so each irrep's pivot
// sequence is the one of the sequential loop.
struct CdState {
  int32_t k[8];          // vectors per irrep
  int32_t k0[8];         // first vector of the current macro iteration
  int32_t gdone[8];      // irrep g has ended its micro iterations
  int32_t steps[8];      // micro iterations of irrep g in this macro iteration
  double tau_mic, pad0;
};

// Qualified list of one macro iteration, grouped by irrep: entries
// [beg[g], beg[g] + cnt[g]) are the qualified pairs of irrep g in Q order
// (slot s of irrep g is entry beg[g] + s).
struct CdQList {
  int32_t beg[8], cnt[8];
};

// C[m][n] = beta C[m][n] + alpha sum_k A[arow(m)][k] B[brow(n)][k].
struct CdGemm {
  const double *A, *B;
  double *C;
  const int32_t *arows, *brows;  // NULL: identity
  int32_t M, N, K, lda, ldb, ldc;
  double alpha, beta;            // C = beta C + alpha A B^T (C not read when beta = 0)
};

// Up to eight independent GEMMs in one launch (one per irrep).
struct CdGemmBatch {
  CdGemm g[8];
  int32_t n, pad0;
};

// Diagonal-block factorisations of one launch (one per irrep).
struct CdDiagBatch {
  double *K[8];
  double *Kinv[8];
  int32_t ld[8], j0[8], w[8];
  int32_t n, pad0;
};

}  // namespace cdcc
