// Split-precision kernels of the (ac|bd) batch assembly for gfx950.
//
// Each operand row x (one (a,c) pair over the Cholesky index) is scaled by a
// power of two sigma and cut into four slices, and the product of two rows is
// a sum of slice products.  Two slice formats:
//
// BF16 (CDCC_MIXED).  sigma >= max|x|, exponent-aligned BF16 slices
//   y = x / sigma = s0 + s1 + s2 + s3 + r,   s_t = m_t 2^-8(t+1), |m_t| <= 256,
// so that |r| <= 2^-33.  Eleven slice products are formed: the ten with
// t + u <= 3 and s2 * s2.  The last one matters beyond its size: on the
// diagonal of the product (both operand rows the same row, and its
// transpose for symmetric vectors) a dropped s_t * s_t is a square, positive
// in every term, and the pair energies weight those diagonal products
// coherently; without s2 * s2 they came out 3-5e-9 too small relative to
// their value (up to 1.1e-8 Eh at |e_ij| = 3.6), with it the bias is gone
// and the first dropped square is s3 * s3, 2^-16 smaller.  The products go
// to three FP32 accumulators, flushed into an FP64 total every 256 K:
//   weight 0, s0 * s0: integer terms of at most 2^16 units of 2^-16, exact in
//     FP32 for 256 K;
//   weight 1, s0 * s1 and s1 * s0 (|m_1| <= 128): terms of at most 2^15 units
//     of 2^-24, two per K, exact for 256 K as well;
//   weights 2 to 4, the other eight: these alone are rounded, at 2^-24 of a
//     sum that is itself about 2^-16 of the result scale (MFMA rounds each
//     accumulation once; sums with bits below the accumulator's last place
//     drift slightly toward zero, so the exact sums are kept apart).
//
// 8-bit digits (CDCC_MIXED_I8).  y = x / sigma = sum_t m_t 2^-(7+8t) + r with
// signed digits m_0 in [-126, 127], m_t in [-128, 127] (t >= 1) and
// |r| <= 2^-32: a base-256 expansion by rounding to nearest, then a carry
// pass that moves a digit of +128 into the one above it (sigma is chosen with
// |128 y| < 126.5, so the leading digit cannot overflow).  The leading digit
// has one bit less than a BF16 slice (BF16 takes it from its exponent), so
// the thirteen products with t + u <= 4 are formed: the dropped ones are then
// below 2^-39 of the row scales and the error is that of the truncation.
// Products of two digits are at most 2^14, so MFMA i32 32x32x32 accumulates
// them exactly; the products of one weight t + u = w share an int32
// accumulator, exact for K <= 32736 (four products of weight 3 per K), and
// longer K runs in segments whose FP64 results are added in order.  The
// Lambda stack's subtracted half is handled by negating the accumulators
// (exact in int32) at its first K block and the total at the end.  The
// accumulators are combined once per segment, in FP64: sum_w acc_w 2^-8w.
//
// The FP64 total is finally scaled by sigma_x sigma_y (exact).
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"

namespace cdcc {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef int i16v __attribute__((ext_vector_type(16)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// MFMA f32 32x32x16 bf16 lane mapping (gfx950): A[i][k] in lane i + 32(k/8),
// element k%8; B[k][j] in lane j + 32(k/8); result register r of lane l is
// D[8(r/4) + 4(l/32) + r%4][l%32].  MFMA i32 32x32x32 i8 has the same row,
// column and result mapping with 16 bytes of K per lane; A and B fragments are
// read with the same K order, so the order inside a 16-byte chunk never
// matters.

__device__ __forceinline__ uint16_t bf16_bits_exact(double v) {
  // v is a small integer times a power of two: exact in float and in BF16
  return uint16_t(__float_as_uint(float(v)) >> 16);
}

// K segment of the 8-bit path: 1023 blocks of 32 (K <= 32736 keeps the
// weight-3 accumulator, four products of at most 2^14 per K, below 2^31).
// Launches whose tiles all fit one segment use the kernel without the
// segment loop (LONGK = false): the loop and its read-modify-write epilogue
// cost registers.
constexpr int kI8SegBlocks = 1023;

// ---------------------------------------------------------------------------
// slice: one workgroup per operand row.  With STAGE the row is first written
// to LDS (dynamic size: halves * np doubles) and read from there twice (for
// the maximum and for the slices); without it, it is read from global memory
// twice.  Rows of a dress job are the Lambda stack built on the fly, exactly
// as the dress kernel builds them:
//   U[P] = B^P_ea - t^P_ea,  U[np + P] = t^P_ea,  t^P_ea = sum_m t_m^e L^P_am
// (without singles, U = B), so the FP64 stack never goes to memory.
// Output per K block: BF16, 16 K x 4 slices x 2 bytes (slice t at bytes
// [32t, 32t + 32)); I8, 32 K x 4 digits x 1 byte (digit t at [32t, 32t + 32)).
// ---------------------------------------------------------------------------
constexpr int kRowPer = 8;    // operand elements per thread in flight while a row is read
constexpr int kDressPer = 4;  // the same for a dressed row (om + 1 loads each)

template <bool STAGE, bool I8>
__global__ __launch_bounds__(256) void slice_kernel(const SliceJob *__restrict__ jobs,
                                                    const int2 *__restrict__ rows,
                                                    const SysPtrs *__restrict__ sp) {
  extern __shared__ double srow[];
  __shared__ double red[4];
  const int2 jr = rows[blockIdx.x];
  const SliceJob J = jobs[jr.x];
  const int row = jr.y;
  const SysPtrs S = sp[J.sys];
  const int K = J.halves * J.np;
  double mx = 0.0;
  const double *src = nullptr;
  if (J.dress) {
    // (STAGE is always set for dress jobs)
    const int a = row / J.ve, e = row - a * J.ve;
    const int va = J.rows / J.ve;
    const CDCC_GLOBAL double *bea = as_global(S.B) + J.b_off + (int64_t(e) * va + a) * J.np;
    if (J.halves == 1) {
      for (int P = threadIdx.x; P < J.np; P += 256) {
        const double u = bea[P];
        srow[P] = u;
        mx = fmax(mx, fabs(u));
      }
    } else {
      const CDCC_GLOBAL double *lam = as_global(S.Bvo) + J.bvo_off + int64_t(a) * J.om * J.np;
      const CDCC_GLOBAL double *t1e = as_global(S.t1) + J.t1_off + e;
      // m outermost over chunks of kDressPer P per thread: the loads of one m
      // are independent, so a chunk costs about om + 1 memory round trips;
      // the sums still run over m in increasing order (P past the end reads
      // a clamped address and is not stored)
      for (int P0 = 0; P0 < J.np; P0 += 256 * kDressPer) {
        int pc[kDressPer];
        double tea[kDressPer], bv[kDressPer];
#pragma unroll
        for (int j = 0; j < kDressPer; ++j) {
          const int P = P0 + 256 * j + int(threadIdx.x);
          pc[j] = P < J.np ? P : J.np - 1;
          bv[j] = bea[pc[j]];
          tea[j] = 0.0;
        }
#pragma unroll 1
        for (int m = 0; m < J.om; ++m) {
          const double c = t1e[int64_t(m) * J.ve];
          const CDCC_GLOBAL double *lm = lam + int64_t(m) * J.np;
#pragma unroll
          for (int j = 0; j < kDressPer; ++j) tea[j] += c * lm[pc[j]];
        }
#pragma unroll
        for (int j = 0; j < kDressPer; ++j) {
          const int P = P0 + 256 * j + int(threadIdx.x);
          if (P < J.np) {
            const double u = bv[j] - tea[j];
            srow[P] = u;
            srow[J.np + P] = tea[j];
            mx = fmax(mx, fmax(fabs(u), fabs(tea[j])));
          }
        }
      }
    }
  } else {
    src = S.opnd + J.src_off + int64_t(row) * K;
    // kRowPer independent loads per thread in flight (clamped addresses past
    // the end, not used)
    for (int k0 = 0; k0 < K; k0 += 256 * kRowPer) {
      double v[kRowPer];
#pragma unroll
      for (int j = 0; j < kRowPer; ++j) {
        const int k = k0 + 256 * j + int(threadIdx.x);
        v[j] = src[k < K ? k : K - 1];
      }
#pragma unroll
      for (int j = 0; j < kRowPer; ++j) {
        const int k = k0 + 256 * j + int(threadIdx.x);
        if (k < K) {
          if (STAGE) srow[k] = v[j];
          mx = fmax(mx, fabs(v[j]));
        }
      }
    }
  }
  // row maximum: within each wave by shuffles, then across the four waves
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  int e = 0;
  if (mx > 0.0) {
    const double f = frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1)  =>  |x| < 2^e
    if (I8 && f >= 253.0 / 256.0) ++e;  // keeps |128 x / sigma| < 126.5
  }
  // x / sigma as ldexp(x, -e): exact, and finite even when the row maximum
  // is subnormal (2^-e itself would overflow there)
  const double sigma = ldexp(1.0, e);
  if (threadIdx.x == 0) S.rowscale[J.scale_off + row] = sigma;
  const int Kh = J.Kp / J.halves;
  unsigned char *__restrict__ dst = S.slices + J.dst_off + int64_t(row) * J.Kp * (I8 ? 4 : 8);
  auto elem = [&](int kp) {
    const int half = kp >= Kh ? 1 : 0;
    const int k = kp - half * Kh;
    return k < J.np ? (STAGE ? srow[half * J.np + k] : src[half * J.np + k]) : 0.0;
  };
  if constexpr (I8) {
    // four consecutive K per thread (Kh is a multiple of 32: never across halves)
#pragma unroll 2
    for (int k4 = threadIdx.x * 4; k4 < J.Kp; k4 += 1024) {
      unsigned w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double v = ldexp(elem(k4 + q), 7 - e);  // 128 x / sigma, |v| < 126.5
        int m[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const double r = floor(v + 0.5);
          m[t] = int(r);
          v = (v - r) * 256.0;  // exact: v - r lies in [-0.5, 0.5)
        }
#pragma unroll
        for (int t = 3; t > 0; --t)
          if (m[t] >= 128) {  // +128 (or +129 after a carry) -> borrow from the digit above
            m[t] -= 256;
            m[t - 1] += 1;
          }
#pragma unroll
        for (int t = 0; t < 4; ++t) w[t] |= (unsigned(m[t]) & 0xffu) << (8 * q);
      }
      unsigned char *o = dst + int64_t(k4 >> 5) * 128 + (k4 & 31);
#pragma unroll
      for (int t = 0; t < 4; ++t) *reinterpret_cast<unsigned *>(o + 32 * t) = w[t];
    }
  } else {
    // four consecutive K per thread (Kh is a multiple of 16: never across
    // halves), one 8-byte store per slice
    uint16_t *d16 = reinterpret_cast<uint16_t *>(dst);
#pragma unroll 2
    for (int k4 = threadIdx.x * 4; k4 < J.Kp; k4 += 1024) {
      unsigned long long w[4] = {0ull, 0ull, 0ull, 0ull};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double y = ldexp(elem(k4 + q), -e);
        const double s0 = rint(y * 256.0) * (1.0 / 256.0);
        double r = y - s0;
        const double s1 = rint(r * 65536.0) * (1.0 / 65536.0);
        r -= s1;
        const double s2 = rint(r * 16777216.0) * (1.0 / 16777216.0);
        r -= s2;
        const double s3 = rint(r * 4294967296.0) * (1.0 / 4294967296.0);
        w[0] |= (unsigned long long)bf16_bits_exact(s0) << (16 * q);
        w[1] |= (unsigned long long)bf16_bits_exact(s1) << (16 * q);
        w[2] |= (unsigned long long)bf16_bits_exact(s2) << (16 * q);
        w[3] |= (unsigned long long)bf16_bits_exact(s3) << (16 * q);
      }
      uint16_t *o = d16 + (k4 >> 4) * 64 + (k4 & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) *reinterpret_cast<unsigned long long *>(o + 16 * t) = w[t];
    }
  }
}

// ---------------------------------------------------------------------------
// assemble (split paths): tile BM x BN, (BM/32) x (BN/WN) waves of 32 x WN
// (WN/32 blocks of 32x32 each).  An LDS row holds one K block (16 K of BF16
// slices or 32 K of 8-bit digits) of all four slices of one operand row (128
// B, eight 16-byte chunks).  Rows are copied from global memory straight into
// LDS (global_load_lds_dwordx4) through a ring of three stages (three LDS
// arrays, the K loop unrolled by three), two K blocks ahead of the MFMAs,
// with one barrier per K block.  A copy instruction writes 64 consecutive
// 16-byte chunks, so the chunk order inside a row is permuted on the source
// side (physical chunk c of row r holds logical chunk c ^ ((r / 2) % 8)): the
// 16 rows a 16-lane group of a fragment read touches then fall on 16
// different 16-byte bank groups of the 256-byte bank width.  Rows past the
// tile edge are read clamped: they only reach results that are never stored.
// The subtracted part of the Lambda stack negates the accumulators (and the
// BF16 running total) at that part's first block, exactly, and the epilogue
// negates the total back; NEG instantiations (launches of a T1-dressed Lambda
// stack) hold that code, the others do not.  (Negating the B fragments instead would not give
// bitwise the same sums: the MFMA's rounding is not symmetric in the sign.)
// ---------------------------------------------------------------------------
template <int BM, int BN, int WN, bool I8, bool LONGK, bool NEG>
__global__ __launch_bounds__(64 * (BM / 32) * (BN / WN)) void assemble_mixed_kernel(
    const P1Desc *__restrict__ descs, const Tile *__restrict__ tiles, Queues Q, int *__restrict__ cnt,
    const SysPtrs *__restrict__ sp, double *__restrict__ xbuf) {
  constexpr int NJ = WN / 32;                  // 32x32 output blocks per wave along N
  constexpr int WAVES_N = BN / WN, WAVES_M = BM / 32;
  constexpr int NW = WAVES_M * WAVES_N;
  constexpr int ROWB = 128;                    // bytes per LDS row
  constexpr int STAGE = (BM + BN) * ROWB;      // bytes per ring stage
  constexpr int NI = (BM + BN) / (8 * NW);     // copy instructions per wave per K block (8 rows each)
  constexpr int KBW = I8 ? 32 : 16;            // K per block
  static_assert((BM + BN) % (8 * NW) == 0, "staging");
  static_assert(I8 || !LONGK, "K segments are an 8-bit-path feature");
  __shared__ __attribute__((aligned(16))) unsigned char st0[STAGE];
  __shared__ __attribute__((aligned(16))) unsigned char st1[STAGE];
  __shared__ __attribute__((aligned(16))) unsigned char st2[STAGE];
  unsigned char *const stage[3] = {st0, st1, st2};
  __shared__ int s_tile;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;
  unsigned dead = 0;

  for (;;) {
    const int t = next_tile(cnt, Q, dead, &s_tile);
    if (t < 0) break;
    const Tile tl = tiles[t];
    const P1Desc D = descs[tl.desc];
    const SysPtrs S = sp[D.sys];
    const int m0 = tl.tm * BM, n0 = tl.tn * BN;
    const int nkb = D.Kp / KBW;
    const int64_t rowstride = int64_t(D.Kp) * (I8 ? 4 : 8);  // bytes per sliced row

    // source of the 16-byte chunk this lane copies in each instruction
    const CDCC_GLOBAL unsigned char *src[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int r = (i * NW + wave) * 8 + (lane >> 3);
      const int part = (lane & 7) ^ ((r >> 1) & 7);
      const unsigned char *base;
      if (r < BM) {
        const int m = m0 + r < D.M ? m0 + r : D.M - 1;
        base = S.slices + D.a_soff + int64_t(m) * rowstride;
      } else {
        const int n = n0 + (r - BM) < D.N ? n0 + (r - BM) : D.N - 1;
        const int dd = n / D.nb, b = n - dd * D.nb;
        base = S.slices + D.b_soff + (int64_t(b) * D.vd + dd) * rowstride;
      }
      src[i] = as_global(base) + part * 16;
    }
    auto issue = [&](unsigned char *st, int kbr) {
      const int kb = kbr < nkb ? kbr : nkb - 1;  // clamped: the last copies are redundant
#pragma unroll
      for (int i = 0; i < NI; ++i)
        lds_copy16(src[i] + int64_t(kb) * ROWB, st + (i * NW + wave) * 8 * ROWB);
    };

    // BF16 state: acc0 the leading product, acc1 the two products of weight
    // one, acc2 the eight of weights two to four
    f16v acc0[NJ], acc1[NJ], acc2[NJ];
    double tot[NJ][16];
    // I8 state: accumulator w holds the products of weight t + u = w
    i16v iacc[5][NJ];
    auto flush = [&]() {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[j][r] += double(acc0[j][r]) + (double(acc1[j][r]) + double(acc2[j][r]));
        acc0[j] = f16v{};
        acc1[j] = f16v{};
        acc2[j] = f16v{};
      }
    };
    // fragment byte offsets inside a stage: slice s of row r is logical
    // chunk 2s + (lane >= 32)
    const int hi = lane >> 5;
    const int arow = wm * 32 + (lane & 31);
    int aoff[4], boff[NJ][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      aoff[s] = arow * ROWB + (((2 * s + hi) ^ ((arow >> 1) & 7)) * 16);
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int brow = BM + wn * WN + j * 32 + (lane & 31);
        boff[j][s] = brow * ROWB + (((2 * s + hi) ^ ((brow >> 1) & 7)) * 16);
      }
    }

    // I8 step in two parts: every fragment of the block is read before the
    // next block's copies are issued (with the reads after the copies, the
    // compiler's LDS-DMA wait tracking falls back to waiting for every copy
    // in flight, which drains the ring), then the thirteen products
    i4v fa[4], fb[NJ][4];
    auto read_i8 = [&](const unsigned char *L) {
#pragma unroll
      for (int s = 0; s < 4; ++s) fa[s] = *reinterpret_cast<const i4v *>(L + aoff[s]);
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int s = 0; s < 4; ++s) fb[j][s] = *reinterpret_cast<const i4v *>(L + boff[j][s]);
    };
    // the thirteen products with t + u <= 4, ordered so that no two
    // consecutive ones share an accumulator
    auto mfma_i8 = [&]() {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
#define CDCC_I8P(t, u) \
  iacc[t + u][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[t], fb[j][u], iacc[t + u][j], 0, 0, 0)
        CDCC_I8P(0, 0);
        CDCC_I8P(0, 1);
        CDCC_I8P(0, 2);
        CDCC_I8P(0, 3);
        CDCC_I8P(1, 3);
        CDCC_I8P(1, 0);
        CDCC_I8P(1, 1);
        CDCC_I8P(1, 2);
        CDCC_I8P(2, 2);
        CDCC_I8P(2, 0);
        CDCC_I8P(2, 1);
        CDCC_I8P(3, 1);
        CDCC_I8P(3, 0);
#undef CDCC_I8P
      }
    };
    auto step = [&](const unsigned char *L, int kb) {
      {
        bf8 a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] = __builtin_bit_cast(bf8, *reinterpret_cast<const u32x4 *>(L + aoff[s]));
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          bf8 b[4];
#pragma unroll
          for (int s = 0; s < 4; ++s)
            b[s] = __builtin_bit_cast(bf8, *reinterpret_cast<const u32x4 *>(L + boff[j][s]));
          acc0[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[0], acc0[j], 0, 0, 0);
          acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[1], acc1[j], 0, 0, 0);
          acc2[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[2], acc2[j], 0, 0, 0);
          acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[0], acc1[j], 0, 0, 0);
          acc2[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[1], acc2[j], 0, 0, 0);
          acc2[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[0], acc2[j], 0, 0, 0);
          acc2[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[3], acc2[j], 0, 0, 0);
          acc2[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[2], acc2[j], 0, 0, 0);
          acc2[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[1], acc2[j], 0, 0, 0);
          acc2[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[3], b[0], acc2[j], 0, 0, 0);
          acc2[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[2], acc2[j], 0, 0, 0);
        }
        if ((kb & 15) == 15 || kb == nkb - 1) flush();  // every 256 K: keep the leading accumulator exact
      }
    };

    // epilogue constants: quotients by vc and nb come from a float
    // reciprocal estimate and are corrected to the exact floor (the estimate
    // is off by at most one)
    const float rvc = 1.0f / float(D.vc), rnb = 1.0f / float(D.nb);
    auto qdiv = [](int x, int d, float rd) {
      int q = int(float(x) * rd);
      while (q * d > x) --q;
      while ((q + 1) * d <= x) ++q;
      return q;
    };
    const CDCC_GLOBAL double *rs = as_global(S.rowscale);
    const int mb = m0 + wm * 32 + 4 * (lane >> 5);

    // K segments (several only in the LONGK kernel)
    const int segb = LONGK ? kI8SegBlocks : (nkb > 0 ? nkb : 1);
    for (int kb0 = 0; kb0 == 0 || kb0 < nkb; kb0 += segb) {
      const int kb1 = nkb < kb0 + segb ? nkb : kb0 + segb;
      if (LONGK && kb0 > 0) __syncthreads();  // every wave is done with the previous segment's stages
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        if constexpr (I8) {
#pragma unroll
          for (int w = 0; w < 5; ++w) iacc[w][j] = i16v{};
        } else {
          acc0[j] = f16v{};
          acc1[j] = f16v{};
          acc2[j] = f16v{};
#pragma unroll
          for (int r = 0; r < 16; ++r) tot[j][r] = 0.0;
        }
      }
      if (kb1 > kb0) {
        issue(stage[0], kb0);
        issue(stage[1], kb0 + 1);
      }
      for (int kb = kb0; kb < kb1; kb += 3) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (kb + q < kb1) {
            // this wave's copies of block kb + q have landed once only the NI
            // copies of the next block are in flight, and its fragment reads of
            // the previous block are done; the barrier then makes every wave's
            // copies visible and frees the stage read in the previous step
            __builtin_amdgcn_s_waitcnt(waitcnt_imm(NI, 0));
            __builtin_amdgcn_s_barrier();
            __asm__ volatile("" ::: "memory");  // no LDS access moves above the barrier
            // first block of the subtracted half: acc <- -acc and, BF16,
            // tot <- -tot (exact; the total is negated back in the epilogue).
            // Here, not between the copies and the fragment reads, so that
            // the reads can still be scheduled ahead of the copies.
            if (NEG && kb + q == D.kneg_blk) {
              if constexpr (I8) {
#pragma unroll
                for (int w = 0; w < 5; ++w)
#pragma unroll
                  for (int j = 0; j < NJ; ++j) iacc[w][j] = -iacc[w][j];
              } else {
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                  acc0[j] = -acc0[j];
                  acc1[j] = -acc1[j];
                  acc2[j] = -acc2[j];
#pragma unroll
                  for (int r = 0; r < 16; ++r) tot[j][r] = -tot[j][r];
                }
              }
            }
            if constexpr (I8) {
              read_i8(stage[q]);
              __asm__ volatile("" ::: "memory");  // fragment reads stay ahead of the copies
              issue(stage[(q + 2) % 3], kb + q + 2);
              mfma_i8();
            } else {
              issue(stage[(q + 2) % 3], kb + q + 2);
              step(stage[q], kb + q);
            }
          }
        }
      }
      // the redundant copies issued past the end must land before the stage
      // memory is reused by the next segment or tile
      __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 0));

      // scale and permuted store (same numbering as the FP64 path); later
      // segments add to what the earlier ones stored (same lane, same element)
      const double sgn = kb1 > D.kneg_blk ? -1.0 : 1.0;
      const double unit = I8 ? 0.5 * sgn * (1.0 / 16384.0) : 0.5 * sgn;  // digit products are in units of 2^-14
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int n = n0 + wn * WN + j * 32 + (lane & 31);
        if (n >= D.N) continue;
        const int dd = qdiv(n, D.nb, rnb), b = n - dd * D.nb;
        const double sb = rs[D.b_scoff + int64_t(b) * D.vd + dd];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int m = mb + 8 * (r >> 2) + (r & 3);
          if (m >= D.M) continue;
          const int am = qdiv(m, D.vc, rvc), c = m - am * D.vc;
          const int a = D.a_first + am;
          if (D.tri && b > a) continue;
          const double sa = rs[D.a_scoff + m];
          const int64_t xcol = D.tri ? (int64_t(a) * (a + 1) / 2 - int64_t(D.ga0) * (D.ga0 + 1) / 2 + b)
                                     : (int64_t(a - D.ga0) * D.vb + b);
          const int64_t xrow = D.xrow0 + int64_t(c) * D.vd + dd;
          double v;
          if constexpr (I8) {
            v = (((double(iacc[4][j][r]) * 0x1p-32 + double(iacc[3][j][r]) * 0x1p-24) +
                  double(iacc[2][j][r]) * 0x1p-16) + double(iacc[1][j][r]) * 0x1p-8) + double(iacc[0][j][r]);
          } else {
            v = tot[j][r];
          }
          double *px = xbuf + D.xoff + xrow * D.ldx + xcol;
          const double x = (unit * (sa * sb)) * v;
          *px = (LONGK && kb0 > 0) ? *px + x : x;
        }
      }
    }
  }
}

// stage_bytes > 0: rows staged in that much dynamic LDS (required for dress
// jobs); 0: rows read from global memory twice.  fmt: 0 BF16, 1 8-bit digits.
hipError_t launch_slice(int fmt, const SliceJob *jobs, const int2 *rows, int nrows, const SysPtrs *sp,
                        int stage_bytes, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  if (fmt == 1) {
    if (stage_bytes > 0)
      slice_kernel<true, true><<<nrows, 256, stage_bytes, s>>>(jobs, rows, sp);
    else
      slice_kernel<false, true><<<nrows, 256, 0, s>>>(jobs, rows, sp);
  } else {
    if (stage_bytes > 0)
      slice_kernel<true, false><<<nrows, 256, stage_bytes, s>>>(jobs, rows, sp);
    else
      slice_kernel<false, false><<<nrows, 256, 0, s>>>(jobs, rows, sp);
  }
  return hipGetLastError();
}

// the four-wave 128 x 128 class of both split formats (kernels_split128.hip)
hipError_t launch_assemble_split128(int fmt, int neg, int grid, const P1Desc *descs, const Tile *tiles,
                                    const Queues &Q, int *cnt, const SysPtrs *sp, double *xbuf, hipStream_t s);
int occupancy_split128(int fmt);

template <bool I8, bool LONGK, bool NEG>
static void launch_assemble_fmt(int cls, int grid, const P1Desc *descs, const Tile *tiles, const Queues &Q, int *cnt,
                                const SysPtrs *sp, double *xbuf, hipStream_t s) {
  switch (cls) {
    case 0: assemble_mixed_kernel<64, 128, 64, I8, LONGK, NEG><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf); break;
    case 1: assemble_mixed_kernel<128, 64, 64, I8, LONGK, NEG><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf); break;
    case 2: assemble_mixed_kernel<128, 128, 64, I8, LONGK, NEG><<<grid, 512, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf); break;
    default: assemble_mixed_kernel<64, 64, 32, I8, LONGK, NEG><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf); break;
  }
}

// longk: some tile of the launch has K > 32736 (8-bit path only); neg: the
// launch assembles a T1-dressed Lambda stack (a subtracted half)
hipError_t launch_assemble_mixed(int fmt, int cls, int longk, int neg, int grid, const P1Desc *descs,
                                 const Tile *tiles, const Queues &Q, int *cnt, const SysPtrs *sp, double *xbuf,
                                 hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  // the four-wave 128 x 128 kernel, except for 8-bit launches with K
  // segments or a T1-dressed Lambda stack
  if (cls == 2 && (fmt == 0 || (!longk && !neg)))
    return launch_assemble_split128(fmt, neg, grid, descs, tiles, Q, cnt, sp, xbuf, s);
  if (fmt == 1) {
    if (longk && neg)
      launch_assemble_fmt<true, true, true>(cls, grid, descs, tiles, Q, cnt, sp, xbuf, s);
    else if (longk)
      launch_assemble_fmt<true, true, false>(cls, grid, descs, tiles, Q, cnt, sp, xbuf, s);
    else if (neg)
      launch_assemble_fmt<true, false, true>(cls, grid, descs, tiles, Q, cnt, sp, xbuf, s);
    else
      launch_assemble_fmt<true, false, false>(cls, grid, descs, tiles, Q, cnt, sp, xbuf, s);
  } else if (neg) {
    launch_assemble_fmt<false, false, true>(cls, grid, descs, tiles, Q, cnt, sp, xbuf, s);
  } else {
    launch_assemble_fmt<false, false, false>(cls, grid, descs, tiles, Q, cnt, sp, xbuf, s);
  }
  return hipGetLastError();
}

template <bool I8>
static int occupancy_fmt(int cls) {
  int n = 0;
  hipError_t e;
  if (cls == 0)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_mixed_kernel<64, 128, 64, I8, false, false>, 256, 0);
  else if (cls == 1)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_mixed_kernel<128, 64, 64, I8, false, false>, 256, 0);
  else if (cls == 2)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_mixed_kernel<128, 128, 64, I8, false, false>, 512, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_mixed_kernel<64, 64, 32, I8, false, false>, 256, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

int occupancy_mixed(int fmt, int cls) {
  if (cls == 2) return occupancy_split128(fmt);
  return fmt == 1 ? occupancy_fmt<true>(cls) : occupancy_fmt<false>(cls);
}

}  // namespace cdcc
