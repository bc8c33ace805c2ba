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

__device__ __forceinline__ uint16_t bf16_bits_exact(double v) {
  // v is a small integer times a power of two: exact in float and in BF16
  return uint16_t(__float_as_uint(float(v)) >> 16);
}

// ---------------------------------------------------------------------------
// slice: one workgroup per operand row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void slice_kernel(const SliceJob *__restrict__ jobs,
                                                    const int2 *__restrict__ rows,
                                                    const SysPtrs *__restrict__ sp) {
  __shared__ double red[256];
  const int2 jr = rows[blockIdx.x];
  const SliceJob J = jobs[jr.x];
  const int row = jr.y;
  const SysPtrs S = sp[J.sys];
  const int K = J.halves * J.np;
  const double *__restrict__ src = S.opnd + J.src_off + int64_t(row) * K;
  double mx = 0.0;
  for (int k = threadIdx.x; k < K; k += 256) mx = fmax(mx, fabs(src[k]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  mx = red[0];
  int e = 0;
  if (mx > 0.0) (void)frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1)  =>  |x| < 2^e
  const double sigma = ldexp(1.0, e), inv = ldexp(1.0, -e);
  if (threadIdx.x == 0) S.rowscale[J.scale_off + row] = sigma;
  const int Kh = J.Kp / J.halves;
  uint16_t *__restrict__ dst = S.slices + J.dst_off + int64_t(row) * J.Kp * 4;
  for (int kp = threadIdx.x; kp < J.Kp; kp += 256) {
    const int half = kp >= Kh ? 1 : 0;
    const int k = kp - half * Kh;
    const double x = k < J.np ? src[half * J.np + k] : 0.0;
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
// slices (128 B + 16 B pad); double-buffered, one barrier per K block.
// ---------------------------------------------------------------------------
template <int BM, int BN, int WN>
__global__ __launch_bounds__(64 * (BM / 32) * (BN / WN)) void assemble_mixed_kernel(
    const P1Desc *__restrict__ descs, const Tile *__restrict__ tiles, Queues Q, int *__restrict__ cnt,
    const SysPtrs *__restrict__ sp, double *__restrict__ xbuf) {
  constexpr int NJ = WN / 32;                  // 32x32 output blocks per wave along N
  constexpr int WAVES_N = BN / WN, WAVES_M = BM / 32;
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  constexpr int ROWB = 144;                    // bytes per LDS row
  constexpr int CPT = (BM + BN) * 8 / NT;      // 16-byte chunks per thread per K block
  constexpr int QA = BM * 8 / NT;              // the first QA chunks of a thread are A rows
  static_assert((BM + BN) * 8 % NT == 0 && BM * 8 % NT == 0, "chunk split");
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][(BM + BN) * ROWB];
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
    const int64_t rowstride = int64_t(D.Kp) * 4;  // uint16 per sliced row

    // source of every staged chunk (clamped row) and whether it is real
    const CDCC_GLOBAL u32x4 *src[CPT];
    bool ok[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int r = (tid >> 3) + (NT / 8) * q, part = tid & 7;
      if (q < QA) {
        const int m = m0 + r;
        ok[q] = m < D.M;
        src[q] = as_global(reinterpret_cast<const u32x4 *>(S.slices + D.a_soff + int64_t(ok[q] ? m : D.M - 1) * rowstride)) + part;
      } else {
        const int n = n0 + (r - BM);
        ok[q] = n < D.N;
        const int nn = ok[q] ? n : D.N - 1;
        const int dd = nn / D.nb, b = nn - dd * D.nb;
        src[q] = as_global(reinterpret_cast<const u32x4 *>(S.slices + D.b_soff + (int64_t(b) * D.vd + dd) * rowstride)) + part;
      }
    }

    f16v acc0[NJ], acc1[NJ];
    double tot[NJ][16];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      acc0[j] = f16v{};
      acc1[j] = f16v{};
#pragma unroll
      for (int r = 0; r < 16; ++r) tot[j][r] = 0.0;
    }

    u32x4 pre[CPT];
    auto gload = [&](int kbr) {
      const int kb = kbr < nkb ? kbr : nkb - 1;  // clamped: the last prefetch is redundant
      const unsigned flip = kb >= D.kneg_blk ? 0x80008000u : 0u;
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        u32x4 v = src[q][int64_t(kb) * 8];
        if (q >= QA) v ^= flip;
        v &= ok[q] ? 0xffffffffu : 0u;
        pre[q] = v;
      }
    };
    auto lstore = [&](int buf) {
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int r = (tid >> 3) + (NT / 8) * q;
        *reinterpret_cast<u32x4 *>(&lds[buf][r * ROWB + (tid & 7) * 16]) = pre[q];
      }
    };
    auto flush = [&]() {
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[j][r] += double(acc0[j][r]) + double(acc1[j][r]);
        acc0[j] = f16v{};
        acc1[j] = f16v{};
      }
    };

    if (nkb > 0) {
      gload(0);
      lstore(0);
    }
    __syncthreads();
    const int arow = wm * 32 + (lane & 31);
    const int koff = (lane >> 5) * 16;
    // chunks of 16 K blocks (256 K); the inner loop is one basic block
    for (int kc = 0; kc < nkb; kc += 16) {
      const int kend = kc + 16 < nkb ? kc + 16 : nkb;
      for (int kb = kc; kb < kend; ++kb) {
        const unsigned char *L = lds[kb & 1];
        gload(kb + 1);
        bf8 a[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
          a[s] = __builtin_bit_cast(bf8, *reinterpret_cast<const u32x4 *>(L + arow * ROWB + s * 32 + koff));
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int brow = BM + wn * WN + j * 32 + (lane & 31);
          bf8 b[4];
#pragma unroll
          for (int s = 0; s < 4; ++s)
            b[s] = __builtin_bit_cast(bf8, *reinterpret_cast<const u32x4 *>(L + brow * ROWB + s * 32 + koff));
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
        lstore((kb + 1) & 1);
        __syncthreads();
      }
      flush();  // 256 K: keep the leading accumulator exact
    }

    // epilogue: scale and permuted store (same numbering as the FP64 path)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int n = n0 + wn * WN + j * 32 + (lane & 31);
        if (m >= D.M || n >= D.N) continue;
        const int am = m / D.vc, c = m - am * D.vc;
        const int a = D.a_first + am;
        const int dd = n / D.nb, b = n - dd * D.nb;
        if (D.tri && b > a) continue;
        const double sa = S.rowscale[D.a_scoff + m];
        const double sb = S.rowscale[D.b_scoff + int64_t(b) * D.vd + dd];
        const int64_t xcol = D.tri ? (int64_t(a) * (a + 1) / 2 - int64_t(D.ga0) * (D.ga0 + 1) / 2 + b)
                                   : (int64_t(a - D.ga0) * D.vb + b);
        const int64_t xrow = D.xrow0 + int64_t(c) * D.vd + dd;
        xbuf[D.xoff + xrow * D.ldx + xcol] = 0.5 * (sa * sb) * tot[j][r];
      }
  }
}

hipError_t launch_slice(const SliceJob *jobs, const int2 *rows, int nrows, const SysPtrs *sp, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  slice_kernel<<<nrows, 256, 0, s>>>(jobs, rows, sp);
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
