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

#include "ladder_types.hpp"

namespace cdcc {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

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
// assemble (mixed): tile BM x BN, 4 waves, each 32 x 64 = two 32x32 blocks.
// LDS rows hold one 16-wide K block of all four slices (128 B + 16 B pad).
// ---------------------------------------------------------------------------
template <int BM, int BN>
__global__ __launch_bounds__(256) void assemble_mixed_kernel(const P1Desc *__restrict__ descs,
                                                             const Tile *__restrict__ tiles, int ntiles,
                                                             int *__restrict__ counter,
                                                             const SysPtrs *__restrict__ sp,
                                                             double *__restrict__ xbuf) {
  constexpr int WAVES_N = BN / 64, WAVES_M = BM / 32;
  static_assert(WAVES_M * WAVES_N == 4, "4 waves of 32x64");
  constexpr int ROWB = 144;                    // bytes per LDS row
  constexpr int CHUNKS = (BM + BN) * 8;        // 16-byte chunks per K block
  constexpr int CPT = CHUNKS / 256;            // chunks per thread
  static_assert(CHUNKS % 256 == 0, "chunk split");
  __shared__ __attribute__((aligned(16))) unsigned char lds[(BM + BN) * ROWB];
  __shared__ int s_tile;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WAVES_N, wn = wave % WAVES_N;

  for (;;) {
    if (tid == 0) s_tile = atomicAdd(counter, 1);
    __syncthreads();
    const int t = s_tile;
    __syncthreads();
    if (t >= ntiles) break;
    const Tile tl = tiles[t];
    const P1Desc D = descs[tl.desc];
    const SysPtrs S = sp[D.sys];
    const int m0 = tl.tm * BM, n0 = tl.tn * BN;
    const int nkb = D.Kp / 16;
    const int64_t rowstride = int64_t(D.Kp) * 4;  // uint16 per sliced row

    // source pointer and sign of every staged chunk
    const uint4 *src[CPT];
    bool neg[CPT];
#pragma unroll
    for (int q = 0; q < CPT; ++q) {
      const int c = tid + 256 * q;
      const int r = c >> 3, part = c & 7;
      src[q] = nullptr;
      neg[q] = false;
      if (r < BM) {
        const int m = m0 + r;
        if (m < D.M) src[q] = reinterpret_cast<const uint4 *>(S.slices + D.a_soff + int64_t(m) * rowstride) + part;
      } else {
        const int n = n0 + (r - BM);
        if (n < D.N) {
          const int dd = n / D.nb, b = n - dd * D.nb;
          src[q] = reinterpret_cast<const uint4 *>(S.slices + D.b_soff + (int64_t(b) * D.vd + dd) * rowstride) + part;
          neg[q] = true;
        }
      }
    }

    f16v acc0[2], acc1[2];
    double tot[2][16];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc0[j] = f16v{};
      acc1[j] = f16v{};
#pragma unroll
      for (int r = 0; r < 16; ++r) tot[j][r] = 0.0;
    }

    uint4 pre[CPT];
    auto gload = [&](int kb) {
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (src[q]) {
          v = src[q][int64_t(kb) * 8];
          if (neg[q] && kb >= D.kneg_blk) {
            v.x ^= 0x80008000u;
            v.y ^= 0x80008000u;
            v.z ^= 0x80008000u;
            v.w ^= 0x80008000u;
          }
        }
        pre[q] = v;
      }
    };
    auto flush = [&]() {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[j][r] += double(acc0[j][r]) + double(acc1[j][r]);
        acc0[j] = f16v{};
        acc1[j] = f16v{};
      }
    };

    if (nkb > 0) gload(0);
    for (int kb = 0; kb < nkb; ++kb) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int c = tid + 256 * q;
        *reinterpret_cast<uint4 *>(lds + (c >> 3) * ROWB + (c & 7) * 16) = pre[q];
      }
      __syncthreads();
      if (kb + 1 < nkb) gload(kb + 1);
      const int arow = wm * 32 + (lane & 31);
      const int koff = (lane >> 5) * 16;
      bf8 a[4], b[2][4];
#pragma unroll
      for (int s = 0; s < 4; ++s)
        a[s] = __builtin_bit_cast(bf8, *reinterpret_cast<const uint4 *>(lds + arow * ROWB + s * 32 + koff));
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int brow = BM + wn * 64 + j * 32 + (lane & 31);
#pragma unroll
        for (int s = 0; s < 4; ++s)
          b[j][s] = __builtin_bit_cast(bf8, *reinterpret_cast<const uint4 *>(lds + brow * ROWB + s * 32 + koff));
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc0[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][0], acc0[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][1], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[j][0], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][2], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[j][1], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[j][0], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0], b[j][3], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1], b[j][2], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[2], b[j][1], acc1[j], 0, 0, 0);
        acc1[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[3], b[j][0], acc1[j], 0, 0, 0);
      }
      if ((kb & 15) == 15) flush();  // 256 K: keep the leading accumulator exact
    }
    flush();

    // epilogue: scale and permuted store (same numbering as the FP64 path)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int n = n0 + wn * 64 + j * 32 + (lane & 31);
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

hipError_t launch_assemble_mixed(int cls, int grid, const P1Desc *descs, const Tile *tiles, int ntiles, int *counter,
                                 const SysPtrs *sp, double *xbuf, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (cls == 0)
    assemble_mixed_kernel<64, 128><<<grid, 256, 0, s>>>(descs, tiles, ntiles, counter, sp, xbuf);
  else
    assemble_mixed_kernel<128, 64><<<grid, 256, 0, s>>>(descs, tiles, ntiles, counter, sp, xbuf);
  return hipGetLastError();
}

}  // namespace cdcc
