// Batched complex GEMM of the mixed-precision propagator on the BF16 matrix cores with
// three-way split operands.
//
// Every FP32 operand entry x is split as x = x0 + x1 + x2 with x0 = bf16(x), x1 = bf16(x - x0),
// x2 = bf16(x - x0 - x1) (each residual is exact in FP32), i.e. 24 significant bits, and a real
// product keeps the six split products whose order is at most 2^-16 of the leading one:
//     a b ~ a0 b0 + (a0 b1 + a1 b0) + (a0 b2 + a1 b1 + a2 b0),
// accumulated in FP32 by v_mfma_f32_16x16x32_bf16.  The dropped terms are below 2^-24 relative,
// the rounding level of the FP32 product it replaces.  A complex product takes the four real
// products re += a.re b.re - a.im b.im, im += a.re b.im + a.im b.re: 24 BF16 MFMAs of 16x16x32
// per 16 x 16 block and 32-deep k chunk, against 32 FP32 MFMAs of 16x16x4 for the same chunk,
// at 16 times the FP32 rate per instruction-cycle.
//
// Tile: 64 x 64 outputs per workgroup of 4 waves (2 x 2 waves of 32 x 32, 2 x 2 blocks of 16 x 16
// each), K staged through LDS 32 deep as complex64, k-contiguous for both operands (A as [m][k],
// B transposed to [n][k]), so that each lane reads the 8 k-consecutive entries of its block row
// (A) or block column (B) as 64 contiguous bytes and splits them into the six bf16 planes
// (re0, re1, re2, im0, im1, im2) in registers with packed conversions.  The staging is
// double-buffered in 68 KB (two workgroups per CU): the next chunk's global loads are issued
// before the current chunk's MFMAs and written to the other buffer after them, one barrier per
// chunk.
// Epilogue and parameters as the other GEMMs of the propagator (GemmParams, role 0): C (complex64
// or complex128) = diag(rs) [alpha A B + beta C + cI I + c1 P1 + c2 P2 + c3 P3] diag(cs), with up
// to four extra outputs from the same product.  A is complex64, B complex64 or complex128
// (rounded to FP32 before the split).
#include "common.h"
#include "kernels.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 64, BN = 64, BK = 32, WM = 32, WN = 32, NT = 256;
constexpr int FM = WM / 16, FN = WN / 16;
constexpr int KP = BK + 2;                // LDS row: 32 complex64 of k plus 16 bytes against bank conflicts

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// Two FP32 values to a packed bf16 pair, round to nearest even (one v_cvt_pk_bf16_f32); element 0
// in the low half.
FT_DEV unsigned cvt2(float a, float b) {
  const f32x2 v = {a, b};
  return __builtin_bit_cast(unsigned, __builtin_convertvector(v, bf16x2));
}
// The three-way split of a pair: h0 = bf16(x), h1 = bf16(x - h0), h2 = bf16(x - h0 - h1), each a
// packed pair (a bf16 widens to FP32 by a 16-bit shift, so the residuals are exact FP32 differences).
FT_DEV void split2(float a, float b, unsigned& h0, unsigned& h1, unsigned& h2) {
  h0 = cvt2(a, b);
  a -= __uint_as_float(h0 << 16);
  b -= __uint_as_float(h0 & 0xffff0000u);
  h1 = cvt2(a, b);
  a -= __uint_as_float(h1 << 16);
  b -= __uint_as_float(h1 & 0xffff0000u);
  h2 = cvt2(a, b);
}

FT_DEV float2 as_f2(float2 v) { return v; }
FT_DEV float2 as_f2(double2 v) { return make_float2((float)v.x, (float)v.y); }

FT_DEV bf16x8 neg8(bf16x8 v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

FT_DEV f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }

template <typename TB, typename TC>
__global__ __launch_bounds__(NT) void zgemm_bf16x6_kernel(GemmParams p) {
  __shared__ __attribute__((aligned(16))) float2 As[2][BM][KP];
  __shared__ __attribute__((aligned(16))) float2 Bs[2][BN][KP];

  int w, tile;
  if (!xcd_walker_tile(blockIdx.x, p.W, p.tiles_m * p.tiles_n, &w, &tile)) return;
  const int tm = tile / p.tiles_n, tn = tile - tm * p.tiles_n;
  const int m0 = tm * BM, n0 = tn * BN;
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int Mr = p.m, Nc = p.n, Kd = p.k;
  const float2* A = (const float2*)p.A + (long long)w * p.sA;
  const TB* B = (const TB*)p.B + (long long)w * p.sB;

  // staging: A row t/4, k 8 (t%4) .. +7 (64 contiguous bytes per thread); B column t%64,
  // k 8 (t/64) .. +7 (consecutive lanes read consecutive columns of one k row)
  const int ar = t >> 2, ak = 8 * (t & 3);
  const int bn = t & 63, bk = 8 * (t >> 6);
  float2 ra[8], rb[8];
  auto load = [&](int kt) {
    const int k0 = kt * BK;
    const int gm = m0 + ar, gn = n0 + bn;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int gk = k0 + ak + e;
      const bool ok = gm < Mr && gk < Kd;
      ra[e] = A[ok ? (long long)gm * p.lda + gk : 0];
      if (!ok) ra[e] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int gk = k0 + bk + e;
      const bool ok = gn < Nc && gk < Kd;
      const TB v = B[ok ? (long long)gk * p.ldb + gn : 0];
      rb[e] = ok ? as_f2(v) : make_float2(0.f, 0.f);
    }
  };
  auto stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      *(float4*)&As[buf][ar][ak + e] = make_float4(ra[e].x, ra[e].y, ra[e + 1].x, ra[e + 1].y);
      *(float4*)&Bs[buf][bn][bk + e] = make_float4(rb[e].x, rb[e].y, rb[e + 1].x, rb[e + 1].y);
    }
  };
  // a fragment: 8 k-consecutive complex64 entries, split into the six bf16 planes (dword d of a
  // plane holds the entries 2d and 2d + 1)
  auto frag = [&](const float2* src, bf16x8 (&out)[6]) {
    u32x4 pl[6];
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      const float4 v = *(const float4*)(src + 2 * d);   // re_2d, im_2d, re_2d+1, im_2d+1
      unsigned h[6];
      split2(v.x, v.z, h[0], h[1], h[2]);
      split2(v.y, v.w, h[3], h[4], h[5]);
#pragma unroll
      for (int q = 0; q < 6; ++q) pl[q][d] = h[q];
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) out[q] = __builtin_bit_cast(bf16x8, pl[q]);
  };

  // the leading split product a0 b0 and the five smaller ones accumulate apart, so that the small
  // terms are not rounded at the scale of the leading one on every chunk
  f32x4 accR[FM][FN], accI[FM][FN], lowR[FM][FN], lowI[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) { accR[i][j][v] = 0.f; accI[i][j][v] = 0.f; lowR[i][j][v] = 0.f; lowI[i][j][v] = 0.f; }

  // 16 x 16 blocks entirely outside the m x n result issue no MFMAs (uniform per wave)
  bool live[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) live[i][j] = (m0 + wr * WM + i * 16 < Mr) && (n0 + wc * WN + j * 16 < Nc);

  const int li = lane & 15, lk = 8 * (lane >> 4);
  const int nk = (Kd + BK - 1) / BK;
  load(0);
  stage(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load(kt + 1);
    bf16x8 a[FM][6], b[FN][6];
#pragma unroll
    for (int i = 0; i < FM; ++i) frag(&As[buf][wr * WM + i * 16 + li][lk], a[i]);
#pragma unroll
    for (int j = 0; j < FN; ++j) frag(&Bs[buf][wc * WN + j * 16 + li][lk], b[j]);
    // the imaginary planes of B negated once: re -= a.im b.im as a.im (-b.im)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int s = 3; s < 6; ++s) b[j][s] = neg8(b[j][s]);
    // split pairs (s, u) with s + u <= 2: the five smaller ones, smallest first, then a0 b0; for
    // each pair every block's two independent first products, then the two dependent second ones
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int s = q == 0 ? 2 : q == 1 ? 1 : q == 2 ? 0 : q == 3 ? 1 : q == 4 ? 0 : 0;
      const int u = q == 0 ? 0 : q == 1 ? 1 : q == 2 ? 2 : q == 3 ? 0 : q == 4 ? 1 : 0;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          if (!live[i][j]) continue;
          f32x4& R = q < 5 ? lowR[i][j] : accR[i][j];
          f32x4& I = q < 5 ? lowI[i][j] : accI[i][j];
          R = mma(a[i][s], b[j][u], R);
          I = mma(a[i][3 + s], b[j][u], I);
        }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          if (!live[i][j]) continue;
          f32x4& R = q < 5 ? lowR[i][j] : accR[i][j];
          f32x4& I = q < 5 ? lowI[i][j] : accI[i][j];
          R = mma(a[i][3 + s], b[j][3 + u], R);     // - a.im b.im (b.im negated)
          I = mma(a[i][s], neg8(b[j][3 + u]), I);   // + a.re b.im
        }
    }
    if (kt + 1 < nk) stage(buf ^ 1);
    __syncthreads();
  }

  TC* C = (TC*)p.C + (long long)w * p.sC;
  const TC* P1 = p.P1 ? (const TC*)p.P1 + (long long)w * p.sP : nullptr;
  const TC* P2 = p.P2 ? (const TC*)p.P2 + (long long)w * p.sP : nullptr;
  const TC* P3 = p.P3 ? (const TC*)p.P3 + (long long)w * p.sP : nullptr;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // output register v of lane l holds row 4 (l/16) + v, column l%16 of the block
        const int gi = m0 + wr * WM + i * 16 + 4 * (lane >> 4) + v;
        const int gj = n0 + wc * WN + j * 16 + li;
        if (gi >= p.mpad || gj >= p.npad) continue;
        const long long off = (long long)gi * p.ldc + gj;
        const bool in = gi < Mr && gj < Nc;
        double2 out = make_double2(0.0, 0.0);
        double2 q1 = out, q2 = out, q3 = out;
        const double2 acc = make_double2((double)accR[i][j][v] + (double)lowR[i][j][v],
                                         (double)accI[i][j][v] + (double)lowI[i][j][v]);
        if (in) {
          const long long offp = (long long)gi * p.ldp + gj;
          if (P1) q1 = to_d2(P1[offp]);
          if (P2) q2 = to_d2(P2[offp]);
          if (P3) q3 = to_d2(P3[offp]);
          const double di = gi == gj ? 1.0 : 0.0;
          out = cscale(acc, p.alpha);
          if (p.beta != 0.0) out = cadd(out, cscale(to_d2(C[off]), p.beta));
          out.x += p.cI * di;
          out = cadd(out, cadd(cscale(q1, p.c1), cadd(cscale(q2, p.c2), cscale(q3, p.c3))));
          if (p.rs) out = cscale(out, p.rs[gi]);
          if (p.cs) out = cscale(out, p.cs[gj]);
        }
        store_c(C + off, out);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (e >= p.nextra) break;
          const GemmOut& o = p.extra[e];
          double2 x = make_double2(0.0, 0.0);
          if (in) {
            x = cscale(acc, o.cacc);
            x.x += o.cI * (gi == gj ? 1.0 : 0.0);
            x = cadd(x, cadd(cscale(q1, o.c1), cadd(cscale(q2, o.c2), cscale(q3, o.c3))));
          }
          store_c((TC*)o.ptr + (long long)w * p.sC + off, x);
        }
      }
}

template <typename TB, typename TC>
hipError_t launch(GemmParams p, hipStream_t s) {
  p.tiles_m = (p.mpad + BM - 1) / BM;
  p.tiles_n = (p.npad + BN - 1) / BN;
  const int blocks = ((p.W + 7) / 8) * 8 * p.tiles_m * p.tiles_n;   // the XCD-aware walker mapping
  if (blocks == 0) return hipSuccess;
  zgemm_bf16x6_kernel<TB, TC><<<blocks, NT, 0, s>>>(p);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_zgemm_bf16x6(const GemmParams& p, bool wide_b, hipStream_t s) {
  if (p.m <= 0 || p.n <= 0) return hipSuccess;
  if (p.mpad < p.m || p.npad < p.n || p.role != 0 || p.opA != 0 || p.opB != 0) return hipErrorInvalidValue;
  return wide_b ? launch<double2, double2>(p, s) : launch<float2, float2>(p, s);
}
