// Split-precision (ac|bd) batch assembly for gfx950, 128 x 128 tiles on four
// waves, for both split formats: BF16 slices and 8-bit digits.
//
// Slices or digits, their products, accumulators and (BF16) flush points are
// those of the schemes of kernels_mixed.hip: per output element the same
// MFMA products reach each accumulator (BF16: in the same order) and the
// FP64 value is formed the same way, so the results are bitwise the same as
// with that file's kernels.  What differs is the schedule:
//  * each wave owns a 64 x 64 block of the tile (2 x 2 MFMA blocks of 32 x 32):
//    16 fragment reads feed 44 BF16 MFMAs per K block of 16, or 52 int8 MFMAs
//    per K block of 32; with one wave per SIMD a wave has 512 registers,
//    enough for the twelve FP32 accumulators and the FP64 totals (BF16) or
//    the twenty int32 accumulators (8-bit), and the fragments;
//  * the fragments of K block k + 1 are read while the MFMAs of block k run,
//    each as soon as the registers it replaces are no longer needed, so no
//    MFMA waits for LDS;
//  * operand rows come from global memory straight into LDS through a ring
//    of four stages, three K blocks ahead, with one barrier per K block;
//  * the subtracted half of the (BF16) Lambda stack negates the accumulators
//    and the running total once, at its first K block (exact), instead of the
//    B fragments of every block; 8-bit Lambda stacks use the eight-wave
//    kernel of kernels_mixed.hip;
//  * the next tile's first copies are issued before this tile's epilogue, and
//    the epilogue takes each element's X offset and scale from row and column
//    tables that were written to LDS when the tile was set up;
//  * the epilogue always issues 64 stores per lane (elements it does not keep
//    go to a sink below the batch buffer), so the next tile's first wait can
//    leave them in flight.
#include <hip/hip_runtime.h>

#include <climits>
#include <type_traits>

#include "kernel_common.hpp"

namespace cdcc {

namespace {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef int i16v __attribute__((ext_vector_type(16)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 128, kBN = 128;              // tile
constexpr int kWaves = 4;                        // 2 x 2 waves of 64 x 64
constexpr int kRowB = 128;                       // LDS bytes per operand row and K block: 16 K x 4 slices x 2 B
constexpr int kStage = (kBM + kBN) * kRowB;      // 32 KiB
constexpr int kNI = (kBM + kBN) / (8 * kWaves);  // copy instructions per wave per K block (8 rows each)

// X offset (element) and power-of-two scale of one tile row or column
struct EpiEntry {
  long long part;
  double s;
};

// One 16-byte chunk per lane from global memory straight into LDS (lane l
// writes bytes [16 l, 16 l + 16) after the wave-uniform LDS byte address
// lds).  Written out rather than through the builtin: the compiler then
// leaves the waits for these copies to the kernel, which knows which stage
// each fragment read touches (with the builtin it sometimes cannot tell the
// stages apart and drains every copy in flight before a read).  The LDS
// address goes in M0; one wait state separates the M0 write from the copy.
__device__ __forceinline__ void lds_dma16(const CDCC_GLOBAL unsigned char *src, unsigned lds) {
  __asm__ volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "{m0}"(lds) : "memory");
}

__device__ __forceinline__ unsigned lds_addr(const unsigned char *p) {
  return unsigned(size_t((const __attribute__((address_space(3))) unsigned char *)(p)));
}

}  // namespace

// MFMA f32 32x32x16 bf16 lane mapping (gfx950): A[i][k] in lane i + 32(k/8),
// element k%8; B[k][j] in lane j + 32(k/8); result register r of lane l is
// D[8(r/4) + 4(l/32) + r%4][l%32].  The int8 32x32x32 MFMA maps A[i][k] to
// lane i + 32(k/16), byte k%16, and its result like the BF16 one, so a lane
// reads the same 16 bytes of a row chunk in both formats.
//
// LDS row layout (as in kernels_mixed.hip): one K block of all four slices or
// digits of an operand row, eight 16-byte chunks; physical chunk c of row r
// holds logical chunk c ^ ((r / 2) % 8), slice or digit s being logical
// chunks 2s and 2s + 1.  I8: 8-bit digits (K blocks of 32); NEG: the launch
// assembles a T1-dressed Lambda stack (with a subtracted half), BF16 only.
template <bool I8, bool NEG>
__global__ __launch_bounds__(256) void assemble_split128_kernel(const P1Desc *__restrict__ descs,
                                                                const Tile *__restrict__ tiles, Queues Q,
                                                                int *__restrict__ cnt,
                                                                const SysPtrs *__restrict__ sp,
                                                                double *__restrict__ xbuf) {
  static_assert(!(I8 && NEG), "8-bit T1-dressed Lambda stacks use the eight-wave kernel");
  constexpr int kKB = I8 ? 32 : 16;  // K per block (one 128-byte row chunk)
  using Frag = typename std::conditional<I8, i4v, bf8>::type;
  __shared__ __attribute__((aligned(16))) unsigned char st0[kStage];
  __shared__ __attribute__((aligned(16))) unsigned char st1[kStage];
  __shared__ __attribute__((aligned(16))) unsigned char st2[kStage];
  __shared__ __attribute__((aligned(16))) unsigned char st3[kStage];
  // epilogue tables of the current and the next tile: entries [0, kBM) are
  // the tile's rows, [kBM, kBM + kBN) its columns.  Row key: a (diagonal
  // irrep block: only b <= a is stored), INT_MAX - 1 (any b), -1 (row past
  // the edge); column key: b, 0 (off the diagonal block), INT_MAX (column
  // past the edge).  An element is stored when its column key <= row key.
  __shared__ EpiEntry etab[2][kBM + kBN];
  __shared__ int ekey[2][kBM + kBN];
  __shared__ int s_tile;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int hi = lane >> 5, l32 = lane & 31;
  unsigned dead = 0;

  // fragment byte offsets inside a stage: A rows wm*64 + 32i + l32, B rows
  // kBM + wn*64 + 32j + l32; the chunk permutation depends on l32 only
  const int sw = (l32 >> 1) & 7;
  int coff[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) coff[s] = ((2 * s + hi) ^ sw) * 16;
  const int abase = (wm * 64 + l32) * kRowB, bbase = (kBM + wn * 64 + l32) * kRowB;

  // per-tile state
  const CDCC_GLOBAL unsigned char *src[kNI];
  int nkb = 0, kneg = 0;

  auto issue = [&](const unsigned char *st, int kb) {
    const unsigned l0 = __builtin_amdgcn_readfirstlane(lds_addr(st) + wave * 8 * kRowB);
#pragma unroll
    for (int i = 0; i < kNI; ++i) lds_dma16(src[i] + int64_t(kb) * kRowB, l0 + i * kWaves * 8 * kRowB);
  };

  // epilogue table entry of this thread (row tid for tid < kBM, else column
  // tid - kBM) for the tile being set up; written to LDS once the tile's
  // first copies have landed
  EpiEntry pe{0, 0.0};
  int pk = 0;

  // Tile setup: copy sources, the copies of the first three K blocks, and the
  // epilogue table entry of this thread.
  auto prepare = [&](int t) {
    const Tile tl = tiles[t];
    const P1Desc D = descs[tl.desc];
    const SysPtrs S = sp[D.sys];
    const int m0 = tl.tm * kBM, n0 = tl.tn * kBN;
    nkb = D.Kp / kKB;
    kneg = D.kneg_blk;
    const int64_t rowstride = int64_t(D.Kp) * (I8 ? 4 : 8);  // bytes per sliced row
#pragma unroll
    for (int i = 0; i < kNI; ++i) {
      const int r = (i * kWaves + wave) * 8 + (lane >> 3);
      const int part = (lane & 7) ^ ((r >> 1) & 7);
      const unsigned char *base;
      if (r < kBM) {
        const int m = m0 + r < D.M ? m0 + r : D.M - 1;  // clamped rows feed results never stored
        base = S.slices + D.a_soff + int64_t(m) * rowstride;
      } else {
        const int n = n0 + (r - kBM) < D.N ? n0 + (r - kBM) : D.N - 1;
        const int dd = n / D.nb, b = n - dd * D.nb;
        base = S.slices + D.b_soff + (int64_t(b) * D.vd + dd) * rowstride;
      }
      src[i] = as_global(base) + part * 16;
    }
    // table entry of this thread: row tid (tid < kBM) or column tid - kBM,
    // computed without branches on tid so that a single load fetches the
    // scale (from a clamped index: entries past the edge are never used) and
    // nothing waits for it before the entry is written to LDS
    const bool isrow = tid < kBM;
    const int m = m0 + tid, n = n0 + tid - kBM;
    const int mc = m < D.M ? m : D.M - 1, nc = n < D.N ? n : D.N - 1;
    const int am = mc / D.vc, c = mc - am * D.vc, a = D.a_first + am;
    const int dd = nc / D.nb, b = nc - dd * D.nb;
    const int64_t acol =
        D.tri ? int64_t(a) * (a + 1) / 2 - int64_t(D.ga0) * (D.ga0 + 1) / 2 : int64_t(a - D.ga0) * D.vb;
    const int64_t sidx = isrow ? D.a_scoff + mc : D.b_scoff + int64_t(b) * D.vd + dd;
    pe.s = as_global(S.rowscale)[sidx];
    pe.part = isrow ? D.xoff + (int64_t(D.xrow0) + int64_t(c) * D.vd) * D.ldx + acol : int64_t(dd) * D.ldx + b;
    pk = isrow ? (m < D.M ? (D.tri ? a : INT_MAX - 1) : -1) : (n < D.N ? (D.tri ? b : 0) : INT_MAX);
    if (nkb > 0) issue(st0, 0);
    if (nkb > 1) issue(st1, 1);
    if (nkb > 2) issue(st2, 2);
  };

  // every lane stores 64 elements per tile, those outside the stored
  // triangle or the tile's edge into its slot of a 64 x 64 sink just below
  // the batch buffer, so that each tile starts with exactly 64 stores in
  // flight after its first copies (the first tile's are 64 stores to
  // distinct sink slots here, which the compiler cannot merge)
  double *const sink = xbuf - 64 * 64 + lane;
  int t = next_tile(cnt, Q, dead, &s_tile);
  int par = 0;
  if (t >= 0) {
    prepare(t);
    __asm__ volatile("" ::: "memory");
#pragma unroll
    for (int e = 0; e < 64; ++e) sink[64 * e] = 0.0;
    __asm__ volatile("" ::: "memory");
  }

  while (t >= 0) {
    // BF16: acc0: s0 s0; acc1: s0 s1 and s1 s0; acc2: the eight products of
    // weights two to four (t + u = 2, 3, and s2 s2); blocks [i][j] of the
    // wave.  8-bit digits: iacc[w] holds the exact int32 sum of the products
    // of weight t + u = w.
    f16v acc0[2][2], acc1[2][2], acc2[2][2];
    double tot[2][2][16];
    i16v iacc[5][2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        if constexpr (I8) {
#pragma unroll
          for (int w = 0; w < 5; ++w) iacc[w][i][j] = i16v{};
        } else {
          acc0[i][j] = f16v{};
          acc1[i][j] = f16v{};
          acc2[i][j] = f16v{};
#pragma unroll
          for (int r = 0; r < 16; ++r) tot[i][j][r] = 0.0;
        }
      }
    Frag fa[2][4], fb[2][4];
    auto read_a = [&](const unsigned char *L, int i) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        fa[i][s] = __builtin_bit_cast(Frag, *reinterpret_cast<const u32x4 *>(L + abase + i * 32 * kRowB + coff[s]));
    };
    auto read_b = [&](const unsigned char *L, int j) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
        fb[j][s] = __builtin_bit_cast(Frag, *reinterpret_cast<const u32x4 *>(L + bbase + j * 32 * kRowB + coff[s]));
    };
    // the products of block (i, j).  BF16, eleven; per accumulator the order
    // is acc0: a0b0; acc1: a0b1, a1b0; acc2: a0b2, a1b1, a2b0, a0b3, a1b2,
    // a2b1, a3b0, a2b2 (consecutive MFMAs on one accumulator need no wait
    // states).  8-bit digits, the thirteen with t + u <= 4 (integer sums:
    // their order does not matter).
    auto sub = [&](int i, int j) {
      if constexpr (I8) {
#define CDCC_Q(t, u) \
  iacc[t + u][i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[i][t], fb[j][u], iacc[t + u][i][j], 0, 0, 0)
        CDCC_Q(0, 0);
        CDCC_Q(0, 1);
        CDCC_Q(0, 2);
        CDCC_Q(0, 3);
        CDCC_Q(1, 3);
        CDCC_Q(1, 0);
        CDCC_Q(1, 1);
        CDCC_Q(1, 2);
        CDCC_Q(2, 2);
        CDCC_Q(2, 0);
        CDCC_Q(2, 1);
        CDCC_Q(3, 1);
        CDCC_Q(3, 0);
#undef CDCC_Q
      } else {
#define CDCC_P(acc, s, u) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[i][s], fb[j][u], acc[i][j], 0, 0, 0)
        CDCC_P(acc0, 0, 0);
        CDCC_P(acc1, 0, 1);
        CDCC_P(acc2, 0, 2);
        CDCC_P(acc1, 1, 0);
        CDCC_P(acc2, 1, 1);
        CDCC_P(acc2, 2, 0);
        CDCC_P(acc2, 0, 3);
        CDCC_P(acc2, 1, 2);
        CDCC_P(acc2, 2, 1);
        CDCC_P(acc2, 3, 0);
        CDCC_P(acc2, 2, 2);
#undef CDCC_P
      }
    };
    // one block at a time, so that few converted values are live at once
    auto flush = [&]() {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int r = 0; r < 16; ++r)
            tot[i][j][r] += double(acc0[i][j][r]) + (double(acc1[i][j][r]) + double(acc2[i][j][r]));
          acc0[i][j] = f16v{};
          acc1[i][j] = f16v{};
          acc2[i][j] = f16v{};
        }
      __builtin_amdgcn_sched_barrier(0);
    };

    // block 0: every copy of this wave has landed, then every wave's; its
    // fragments go to registers.  The 64 stores of the previous epilogue
    // (or of the sink) were issued after this tile's scale load and first
    // copies, and vector memory operations complete in issue order, so at
    // most 63 in flight leaves the load and the copies of blocks 0-2 done
    // while the stores drain.  The epilogue table of this tile goes to slot
    // par (the previous tile's epilogue, which other waves may still be in,
    // reads the other slot).
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(63, 0));
    etab[par][tid] = pe;
    ekey[par][tid] = pk;
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
    read_a(st0, 0);
    read_a(st0, 1);
    read_b(st0, 0);
    read_b(st0, 1);

    for (int k0 = 0; k0 < nkb; k0 += 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = k0 + q;
        if (k < nkb) {
          // this wave's copies of block k + 1 have landed once only those of
          // block k + 2 may be in flight (blocks 1 and 2 have landed by the
          // tile's first wait); after the barrier every wave's have, and
          // every wave is done with block k - 1 (its stage is refilled below)
          if (k >= 2) {
            if (k + 2 < nkb)
              __builtin_amdgcn_s_waitcnt(waitcnt_imm(kNI, 15));
            else
              __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 15));
          }
          __builtin_amdgcn_s_barrier();
          __asm__ volatile("" ::: "memory");  // no LDS access moves above the barrier
          if (k + 3 < nkb) issue(q == 0 ? st3 : q == 1 ? st0 : q == 2 ? st1 : st2, k + 3);
          if (NEG && k == kneg) {
            // first block of the subtracted half: negate (exact), and the
            // total is negated back in the epilogue
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 2; ++j) {
                acc0[i][j] = -acc0[i][j];
                acc1[i][j] = -acc1[i][j];
                acc2[i][j] = -acc2[i][j];
#pragma unroll
                for (int r = 0; r < 16; ++r) tot[i][j][r] = -tot[i][j][r];
              }
          }
          // fragments of block k + 1 replace those of block k as soon as
          // these are no longer needed: B0 after blocks (0,0) and (1,0), A0
          // after (0,1), A1 and B1 at the end; each is first used 11 to 33
          // MFMAs after its read
          const unsigned char *nx = q == 0 ? st1 : q == 1 ? st2 : q == 2 ? st3 : st0;
          __builtin_amdgcn_sched_barrier(0);
          sub(0, 0);
          __builtin_amdgcn_sched_barrier(0);
          sub(1, 0);
          __builtin_amdgcn_sched_barrier(0);
          read_b(nx, 0);
          __builtin_amdgcn_sched_barrier(0);
          sub(0, 1);
          __builtin_amdgcn_sched_barrier(0);
          read_a(nx, 0);
          __builtin_amdgcn_sched_barrier(0);
          sub(1, 1);
          __builtin_amdgcn_sched_barrier(0);
          // the eight reads issued above are done by now; waiting for them
          // here keeps at most eight reads in flight across the barrier, so
          // the next block's MFMAs wait only for the ones they use
          __builtin_amdgcn_s_waitcnt(waitcnt_imm(63, 0));
          read_a(nx, 1);
          read_b(nx, 1);
          __builtin_amdgcn_sched_barrier(0);
          if constexpr (!I8) {
            if ((k & 15) == 15 || k == nkb - 1) flush();  // every 256 K: keeps acc0 and acc1 exact
          }
        }
      }
    }

    if constexpr (I8) {
      // the digit sums in FP64, one block at a time (one rounding per
      // element: every term but the last sum is exact); here, before the
      // next tile is set up, so that its copy addresses are not live beside
      // the twenty accumulators
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int r = 0; r < 16; ++r)
            tot[i][j][r] = (((double(iacc[4][i][j][r]) * 0x1p-32 + double(iacc[3][i][j][r]) * 0x1p-24) +
                             double(iacc[2][i][j][r]) * 0x1p-16) +
                            double(iacc[1][i][j][r]) * 0x1p-8) +
                           double(iacc[0][i][j][r]);
        }
      __builtin_amdgcn_sched_barrier(0);
    }

    // every wave is done with the stages (the barrier of the claim), then
    // the next tile's first copies go out before this tile's stores
    const int tn = next_tile(cnt, Q, dead, &s_tile);
    const int nkb_c = nkb, kneg_c = kneg;
    if (tn >= 0) prepare(tn);
    __asm__ volatile("" ::: "memory");  // the epilogue stays after the next tile's copies

    // negated total of a Lambda stack; digit products are in units of 2^-14
    const double unit = (kneg_c < nkb_c ? -0.5 : 0.5) * (I8 ? 1.0 / 16384.0 : 1.0);
    EpiEntry ce[2];
    int ck[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = wn * 64 + j * 32 + l32;
      ce[j] = etab[par][kBM + col];
      ck[j] = ekey[par][kBM + col];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wm * 64 + i * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
        const EpiEntry re = etab[par][row];
        const int rk = ekey[par][row];
#pragma unroll
        for (int j = 0; j < 2; ++j)
        {
          double *const dst = ck[j] <= rk ? xbuf + (re.part + ce[j].part) : sink;
          *dst = (unit * (re.s * ce[j].s)) * tot[i][j][r];
        }
      }
    __asm__ volatile("" ::: "memory");  // and before the next tile's table writes
    t = tn;
    par ^= 1;
  }
}

// fmt: 0 split-BF16, 1 8-bit digits (every tile of the launch has K <= 32736,
// so its int32 sums stay exact); neg: a T1-dressed Lambda stack, split-BF16
// only (the 8-bit form negates twenty int32 accumulators in its K loop, and
// with them the compiler runs out of registers and spills)
hipError_t launch_assemble_split128(int fmt, int neg, int grid, const P1Desc *descs, const Tile *tiles,
                                    const Queues &Q, int *cnt, const SysPtrs *sp, double *xbuf, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (fmt == 1 && neg) return hipErrorInvalidValue;
  if (fmt == 1)
    assemble_split128_kernel<true, false><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf);
  else if (neg)
    assemble_split128_kernel<false, true><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf);
  else
    assemble_split128_kernel<false, false><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf);
  return hipGetLastError();
}

int occupancy_split128(int fmt) {
  int n = 0;
  const hipError_t e = fmt == 1 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                      &n, assemble_split128_kernel<true, false>, 256, 0)
                                : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                      &n, assemble_split128_kernel<false, false>, 256, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace cdcc
