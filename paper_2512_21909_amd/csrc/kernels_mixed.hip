// Split-BF16 kernels of the (ac|bd) batch assembly for gfx950 (mixed path).
//
// Each operand row x (one (a,c) pair over the Cholesky index) is scaled by a
// power of two sigma >= max|x| and cut into four exponent-aligned BF16 slices
//   y = x / sigma = s0 + s1 + s2 + s3 + r,   s_t = m_t 2^-8(t+1), |m_t| <= 256,
// so that |r| <= 2^-33.  The product of two rows is the sum of the ten slice
// products with t + u <= 3.  The leading product s0 * s0 has 16-bit integer
// terms in units of 2^-16: accumulated in FP32 on MFMA it is exact for up to
// 256 terms, so it is flushed into an FP64 total every 256 K.  The nine
// lower-order products go to a second FP32 accumulator (their rounding is
// 2^-32 relative to the result scale) and are flushed at the same points.
// The FP64 total is finally scaled by sigma_x sigma_y (exact).
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"

namespace cdcc {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// MFMA f32 32x32x16 bf16 lane mapping (gfx950): A[i][k] in lane i + 32(k/8),
// element k%8; B[k][j] in lane j + 32(k/8); result register r of lane l is
// D[8(r/4) + 4(l/32) + r%4][l%32].

// s_waitcnt immediate (gfx9 encoding: vmcnt in bits 3:0 and 15:14, expcnt in
// 6:4, lgkmcnt in 11:8): wait for vmcnt <= v and lgkmcnt <= l.
constexpr int waitcnt_imm(int v, int l) { return (v & 15) | ((v >> 4) << 14) | (7 << 4) | (l << 8); }

// One 16-byte chunk per lane from global memory straight into LDS: lane l
// writes bytes [16 l, 16 l + 16) after the wave-uniform LDS pointer dst.
// The copies are counted on vmcnt; the caller waits for them with explicit
// s_waitcnt vmcnt and a barrier.
__device__ __forceinline__ void lds_copy16(const CDCC_GLOBAL unsigned char *src, unsigned char *dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(dst), 16, 0, 0);
}

__device__ __forceinline__ uint16_t bf16_bits_exact(double v) {
  // v is a small integer times a power of two: exact in float and in BF16
  return uint16_t(__float_as_uint(float(v)) >> 16);
}

// ---------------------------------------------------------------------------
// slice: one workgroup per operand row.  With STAGE the row is first written
// to LDS (dynamic size: halves * np doubles) and read from there twice (for
// the maximum and for the slices); without it, it is read from global memory
// twice.  Rows of a dress job are the Lambda stack built on the fly, exactly
// as the dress kernel builds them:
//   U[P] = B^P_ea - t^P_ea,  U[np + P] = t^P_ea,  t^P_ea = sum_m t_m^e L^P_am
// (without singles, U = B), so the FP64 stack never goes to memory.
// ---------------------------------------------------------------------------
template <bool STAGE>
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
#pragma unroll 2
      for (int P = threadIdx.x; P < J.np; P += 256) {
        double tea = 0.0;
        for (int m = 0; m < J.om; ++m) tea += t1e[int64_t(m) * J.ve] * lam[int64_t(m) * J.np + P];
        const double u = bea[P] - tea;
        srow[P] = u;
        srow[J.np + P] = tea;
        mx = fmax(mx, fmax(fabs(u), fabs(tea)));
      }
    }
  } else {
    src = S.opnd + J.src_off + int64_t(row) * K;
#pragma unroll 4
    for (int k = threadIdx.x; k < K; k += 256) {
      const double u = src[k];
      if (STAGE) srow[k] = u;
      mx = fmax(mx, fabs(u));
    }
  }
  // row maximum: within each wave by shuffles, then across the four waves
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  int e = 0;
  if (mx > 0.0) (void)frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1)  =>  |x| < 2^e
  const double sigma = ldexp(1.0, e), inv = ldexp(1.0, -e);
  if (threadIdx.x == 0) S.rowscale[J.scale_off + row] = sigma;
  const int Kh = J.Kp / J.halves;
  uint16_t *__restrict__ dst = S.slices + J.dst_off + int64_t(row) * J.Kp * 4;
#pragma unroll 4
  for (int kp = threadIdx.x; kp < J.Kp; kp += 256) {
    const int half = kp >= Kh ? 1 : 0;
    const int k = kp - half * Kh;
    const double x = k < J.np ? (STAGE ? srow[half * J.np + k] : src[half * J.np + k]) : 0.0;
    const double y = x * inv;
    const double s0 = rint(y * 256.0) * (1.0 / 256.0);
    double r = y - s0;
    const double s1 = rint(r * 65536.0) * (1.0 / 65536.0);
    r -= s1;
    const double s2 = rint(r * 16777216.0) * (1.0 / 16777216.0);
    r -= s2;
    const double s3 = rint(r * 4294967296.0) * (1.0 / 4294967296.0);
    uint16_t *o = dst + (kp >> 4) * 64 + (kp & 15);
    o[0] = bf16_bits_exact(s0);
    o[16] = bf16_bits_exact(s1);
    o[32] = bf16_bits_exact(s2);
    o[48] = bf16_bits_exact(s3);
  }
}

// ---------------------------------------------------------------------------
// assemble (mixed): tile BM x BN, (BM/32) x (BN/WN) waves of 32 x WN (WN/32
// blocks of 32x32 each).  An LDS row holds one 16-wide K block of all four
// slices of one operand row (128 B, eight 16-byte chunks).  Rows are copied
// from global memory straight into LDS (global_load_lds_dwordx4) through a
// ring of three stages (three LDS arrays, the K loop unrolled by three),
// two K blocks ahead of the MFMAs, with one barrier per K block.  A copy instruction writes 64 consecutive 16-byte chunks, so
// the chunk order inside a row is permuted on the source side (physical
// chunk c of row r holds logical chunk c ^ ((r / 2) % 8)): the 16 rows a
// 16-lane group of a fragment read touches then fall on 16 different
// 16-byte bank groups of the 256-byte bank width.  Rows past the tile edge are read
// clamped: they only reach results that are never stored.  The sign of the
// subtracted part of the Lambda stack is applied to the B fragments.
// ---------------------------------------------------------------------------
template <int BM, int BN, int WN>
__global__ __launch_bounds__(64 * (BM / 32) * (BN / WN)) void assemble_mixed_kernel(
    const P1Desc *__restrict__ descs, const Tile *__restrict__ tiles, Queues Q, int *__restrict__ cnt,
    const SysPtrs *__restrict__ sp, double *__restrict__ xbuf) {
  constexpr int NJ = WN / 32;                  // 32x32 output blocks per wave along N
  constexpr int WAVES_N = BN / WN, WAVES_M = BM / 32;
  constexpr int NW = WAVES_M * WAVES_N;
  constexpr int ROWB = 128;                    // bytes per LDS row
  constexpr int STAGE = (BM + BN) * ROWB;      // bytes per ring stage
  constexpr int NI = (BM + BN) / (8 * NW);     // copy instructions per wave per K block (8 rows each)
  static_assert((BM + BN) % (8 * NW) == 0, "staging");
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
    const int nkb = D.Kp / 16;
    const int64_t rowstride = int64_t(D.Kp) * 8;  // bytes per sliced row

    // source of the 16-byte chunk this lane copies in each instruction
    const CDCC_GLOBAL unsigned char *src[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int r = (i * NW + wave) * 8 + (lane >> 3);
      const int part = (lane & 7) ^ ((r >> 1) & 7);
      const unsigned char *base;
      if (r < BM) {
        const int m = m0 + r < D.M ? m0 + r : D.M - 1;
        base = reinterpret_cast<const unsigned char *>(S.slices + D.a_soff) + int64_t(m) * rowstride;
      } else {
        const int n = n0 + (r - BM) < D.N ? n0 + (r - BM) : D.N - 1;
        const int dd = n / D.nb, b = n - dd * D.nb;
        base = reinterpret_cast<const unsigned char *>(S.slices + D.b_soff) + (int64_t(b) * D.vd + dd) * rowstride;
      }
      src[i] = as_global(base) + part * 16;
    }
    auto issue = [&](unsigned char *st, int kbr) {
      const int kb = kbr < nkb ? kbr : nkb - 1;  // clamped: the last copies are redundant
#pragma unroll
      for (int i = 0; i < NI; ++i)
        lds_copy16(src[i] + int64_t(kb) * ROWB, st + (i * NW + wave) * 8 * ROWB);
    };

    f16v acc0[NJ], acc1[NJ];
    double tot[NJ][16];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      acc0[j] = f16v{};
      acc1[j] = f16v{};
#pragma unroll
      for (int r = 0; r < 16; ++r) tot[j][r] = 0.0;
    }
    auto flush = [&]() {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[j][r] += double(acc0[j][r]) + double(acc1[j][r]);
        acc0[j] = f16v{};
        acc1[j] = f16v{};
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

    auto step = [&](const unsigned char *L, int kb) {
      const unsigned flip = kb >= D.kneg_blk ? 0x80008000u : 0u;
      bf8 a[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) a[s] = __builtin_bit_cast(bf8, *reinterpret_cast<const u32x4 *>(L + aoff[s]));
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        bf8 b[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
          b[s] = __builtin_bit_cast(bf8, *reinterpret_cast<const u32x4 *>(L + boff[j][s]) ^ flip);
        acc0[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[0], acc0[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[1], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[0], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[2], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[1], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[0], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[3], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[2], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[1], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[3], b[0], acc1[j], 0, 0, 0);
      }
      if ((kb & 15) == 15 || kb == nkb - 1) flush();  // every 256 K: keep the leading accumulator exact
    };

    if (nkb > 0) {
      issue(stage[0], 0);
      issue(stage[1], 1);
    }
    for (int kb = 0; kb < nkb; kb += 3) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (kb + q < nkb) {
          // this wave's copies of block kb + q have landed once only the NI
          // copies of the next block are in flight, and its fragment reads of
          // the previous block are done; the barrier then makes every wave's
          // copies visible and frees the stage read in the previous step
          __builtin_amdgcn_s_waitcnt(waitcnt_imm(NI, 0));
          __builtin_amdgcn_s_barrier();
          __asm__ volatile("" ::: "memory");  // no LDS access moves above the barrier
          issue(stage[(q + 2) % 3], kb + q + 2);
          step(stage[q], kb + q);
        }
      }
    }
    // the redundant copies issued past the end must land before the stage
    // memory is reused by the next tile
    __builtin_amdgcn_s_waitcnt(waitcnt_imm(0, 0));

    // epilogue: scale and permuted store (same numbering as the FP64 path).
    // Quotients by vc and nb come from a float reciprocal estimate and are
    // corrected to the exact floor (the estimate is off by at most one).
    const float rvc = 1.0f / float(D.vc), rnb = 1.0f / float(D.nb);
    auto qdiv = [](int x, int d, float rd) {
      int q = int(float(x) * rd);
      while (q * d > x) --q;
      while ((q + 1) * d <= x) ++q;
      return q;
    };
    const CDCC_GLOBAL double *rs = as_global(S.rowscale);
    const int mb = m0 + wm * 32 + 4 * (lane >> 5);
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
        xbuf[D.xoff + xrow * D.ldx + xcol] = 0.5 * (sa * sb) * tot[j][r];
      }
    }
  }
}

// stage_bytes > 0: rows staged in that much dynamic LDS (required for dress
// jobs); 0: rows read from global memory twice.
hipError_t launch_slice(const SliceJob *jobs, const int2 *rows, int nrows, const SysPtrs *sp, int stage_bytes,
                        hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  if (stage_bytes > 0)
    slice_kernel<true><<<nrows, 256, stage_bytes, s>>>(jobs, rows, sp);
  else
    slice_kernel<false><<<nrows, 256, 0, s>>>(jobs, rows, sp);
  return hipGetLastError();
}

hipError_t launch_assemble_mixed(int cls, int grid, const P1Desc *descs, const Tile *tiles, const Queues &Q,
                                 int *cnt, const SysPtrs *sp, double *xbuf, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  switch (cls) {
    case 0: assemble_mixed_kernel<64, 128, 64><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf); break;
    case 1: assemble_mixed_kernel<128, 64, 64><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf); break;
    case 2: assemble_mixed_kernel<128, 128, 64><<<grid, 512, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf); break;
    default: assemble_mixed_kernel<64, 64, 32><<<grid, 256, 0, s>>>(descs, tiles, Q, cnt, sp, xbuf); break;
  }
  return hipGetLastError();
}

int occupancy_mixed(int cls) {
  int n = 0;
  hipError_t e;
  if (cls == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_mixed_kernel<64, 128, 64>, 256, 0);
  else if (cls == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_mixed_kernel<128, 64, 64>, 256, 0);
  else if (cls == 2) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_mixed_kernel<128, 128, 64>, 512, 0);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, assemble_mixed_kernel<64, 64, 32>, 256, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

}  // namespace cdcc
