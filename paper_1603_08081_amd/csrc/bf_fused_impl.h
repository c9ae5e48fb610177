#pragma once
// Fused shiftable bilateral filter for gfx950 (one image per launch).
//
// Computes eq. (9) of the paper through Algorithm 1 in its real (cos/sin)
// form: with theta_k(j) = k w f(j), w = pi / T, and c0 = T / 2,
//   P(i) = sum_k d_k [cos theta_k(i) * (w * C_k)(i) + sin theta_k(i) * (w * S_k)(i)]  (Q)
//   with C_k = cos theta_k, S_k = sin theta_k for the denominator and
//   C_k = (f - c0) cos theta_k, S_k = (f - c0) sin theta_k for the numerator;
//   the k = 0 term is d_0 (w * (f - c0)) for P and d_0 sum(w) for Q, and the
//   output is P / Q + c0.  Summing the harmonics +k and -k of eq. (4) with
//   c_{+-k} = d_k / 2 gives exactly this real form (relation after eq. (6)).
//
// Work decomposition.  A workgroup (4 waves) owns a 64-column x TH-row output
// tile; wave w owns the 16-column strip [X0 + 16w, X0 + 16w + 16).  For each
// harmonic k the workgroup walks down the tile in 16-row steps:
//   1. modulate 16 input rows (the strip plus a W-column halo) into LDS --
//      each input pixel is modulated once per step and shared by the 4 waves;
//   2. row pass: one MFMA banded-Toeplitz product per 32 (16-bit) or 4
//      (fp32) input columns, with the Toeplitz weights held in registers;
//      the 16x16 fp32 result of each plane stays in registers (a ring of the
//      last NT row tiles);
//   3. column pass: once the ring spans 16 output rows plus the W-row halos,
//      a second Toeplitz product runs straight from the ring registers (the
//      MFMA output layout of the row pass is, up to a fixed permutation of the
//      contraction index that the weights absorb, the input layout of the
//      column pass), so row-filtered planes never touch LDS or HBM;
//   4. demodulate at the 16x16 output pixels and accumulate P, Q in fp32
//      registers.
// The phase e^{i theta} is read from a 2T-entry table of cos/sin(pi m / T)
// built per workgroup in float64 and rounded once; for integer gray levels
// the index k f mod 2T is exact.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "bf_internal.h"
#include "bf_fused.h"

namespace bf {
namespace fused_detail {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 b16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 b16x4 __attribute__((ext_vector_type(4)));

template <int PREC>
struct Planes;

template <>
struct Planes<BF_PLANES_FP32> {
  using E = float;
  static __device__ __forceinline__ float round(float x) { return x; }
};

template <>
struct Planes<BF_PLANES_FP16> {
  using E = _Float16;
  using V8 = f16x8;
  using V4 = f16x4;
  static __device__ __forceinline__ float round(float x) { return (float)(_Float16)x; }
  static __device__ __forceinline__ f32x4 mma(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Planes<BF_PLANES_BF16> {
  using E = __bf16;
  using V8 = b16x8;
  using V4 = b16x4;
  static __device__ __forceinline__ float round(float x) { return (float)(__bf16)x; }
  static __device__ __forceinline__ f32x4 mma(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

// half-sample symmetric fold, then clamp (the clamp only matters for pixels
// whose outputs are never stored)
__device__ __forceinline__ int fold(int i, int n) {
  i = (i < 0) ? -i - 1 : i;
  i = (i >= n) ? 2 * n - i - 1 : i;
  return min(max(i, 0), n - 1);
}

__device__ __forceinline__ float fma_acc(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_acc(double a, double b, double c) { return fma(a, b, c); }

struct PhaseTab {
  const float2* lut;  // cos, sin of pi m / T, m = 0..2T-1
  float two_t, inv_two_t, inv_t;
  int n_lut;          // 2T
};

// cos and sin of k w f with w = pi / T
template <bool INTEGER>
__device__ __forceinline__ void phase(float kf, float f, const PhaseTab& pt, float& c, float& s) {
  if constexpr (INTEGER) {
    const float p = kf * f;  // exact for integer f
    const float q = floorf(p * pt.inv_two_t);
    float m = fmaf(-pt.two_t, q, p);
    m = (m >= pt.two_t) ? m - pt.two_t : m;
    m = (m < 0.f) ? m + pt.two_t : m;
    const float2 v = pt.lut[min(max((int)m, 0), pt.n_lut - 1)];  // clamp: non-finite input
    c = v.x;
    s = v.y;
  } else {
    // k f = k floor(f) + k frac(f): the integer part indexes the table
    // exactly, the remaining fraction r in [0, 1) is applied as a rotation
    const float fi = floorf(f);
    const float pf = kf * (f - fi);
    const float n2 = floorf(pf);
    const float r = pf - n2;
    const float p = fmaf(kf, fi, n2);
    const float q = floorf(p * pt.inv_two_t);
    float m = fmaf(-pt.two_t, q, p);
    m = (m >= pt.two_t) ? m - pt.two_t : m;
    m = (m < 0.f) ? m + pt.two_t : m;
    const float2 v = pt.lut[min(max((int)m, 0), pt.n_lut - 1)];
    float sr, cr;
    sincospif(r * pt.inv_t, &sr, &cr);
    c = v.x * cr - v.y * sr;
    s = v.y * cr + v.x * sr;
  }
}

template <int PREC, int NT, int TH, bool INTEGER>
__global__ void __launch_bounds__(256) fused_kernel(const JobDesc job) {
  using PT = Planes<PREC>;
  using E = typename PT::E;
  constexpr bool F32 = (PREC == BF_PLANES_FP32);
  constexpr int KS = (NT + 1) / 2;       // 32-column contraction steps
  constexpr int LWU = 48 + 32 * KS;      // LDS columns used per plane row
  constexpr int LW = F32 ? LWU + 4 : LWU + 8;  // padded row (bank spread, 16 B aligned)
  constexpr int NJ = TH / 16;            // output row tiles per workgroup
  constexpr int NS = NJ + NT - 1;        // 16-row steps per harmonic

  __shared__ __attribute__((aligned(16))) E planes[2][4][16][LW];
  __shared__ float w1s[2 * BF_MAX_W + 1];
  extern __shared__ float2 lut[];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, n16 = lane & 15;
  const int X0 = blockIdx.x * kTileCols, Y0 = blockIdx.y * TH;
  const int x0 = X0 + 16 * wave;
  const int W = job.W, T = job.T, K = job.K;
  const int H = job.height, Wd = job.width;
  const float* __restrict__ src = job.src;
  const int sp = job.src_pitch;
  const float c0 = job.c0;

  for (int m = tid; m < 2 * T; m += 256) {
    double s, c;
    sincospi((double)m / (double)T, &s, &c);
    lut[m] = make_float2((float)c, (float)s);
  }
  for (int t = tid; t <= 2 * W; t += 256) w1s[t] = job.w1[t];
  __syncthreads();

  auto wq = [&](int dd) -> float { return (dd >= -W && dd <= W) ? PT::round(w1s[dd + W]) : 0.f; };

  // Toeplitz operands.  Row pass: B[k][n] = w(input col - output col) with the
  // input col of contraction slot k counted from x0 - W.  Column pass: the
  // contraction slot (lane group g, element e) holds row 4g + (e & 3) of ring
  // tile 2ks + (e >> 2) (16-bit) or row 4g + i of ring tile t (fp32).
  using BrowT = std::conditional_t<F32, float, typename std::conditional_t<F32, Planes<BF_PLANES_FP16>, PT>::V8>;
  constexpr int NBR = F32 ? 8 * KS : KS;
  BrowT brow[NBR];
  float bcol32[F32 ? NT : 1][4];
  BrowT bcol16[F32 ? 1 : KS];
  if constexpr (F32) {
    for (int s4 = 0; s4 < NBR; ++s4) brow[s4] = wq(4 * s4 + g - W - n16);
    for (int t = 0; t < NT; ++t)
      for (int i = 0; i < 4; ++i) bcol32[t][i] = wq(16 * t + 4 * g + i - W - n16);
  } else {
    for (int ks = 0; ks < KS; ++ks)
      for (int e = 0; e < 8; ++e) {
        brow[ks][e] = (E)wq(32 * ks + 8 * g + e - W - n16);
        bcol16[ks][e] = (E)wq(16 * (2 * ks + (e >> 2)) + 4 * g + (e & 3) - W - n16);
      }
  }
  const int nks4 = (16 + 2 * W + 3) / 4;  // fp32 row-pass steps with nonzero weights
  // fp32 planes accumulate P and Q in float64 (see the column pass below);
  // 16-bit planes are limited by their own rounding and accumulate in float32
  using Acc = std::conditional_t<F32, double, float>;
  double wsum = 0.0;
  for (int t = -W; t <= W; ++t) wsum += (double)wq(t);
  const Acc q0 = (Acc)(job.d[0] * wsum * wsum);

  // gray levels at this lane's output pixels: row Y0 + 16 j + n16, cols x0 + 4 g + i
  float fo[NJ][4];
  for (int j = 0; j < NJ; ++j)
    for (int i = 0; i < 4; ++i) {
      const int yy = min(Y0 + 16 * j + n16, H - 1), xx = min(x0 + 4 * g + i, Wd - 1);
      fo[j][i] = src[(size_t)yy * sp + xx];
    }
  Acc P[NJ][4], Q[NJ][4];
  for (int j = 0; j < NJ; ++j)
    for (int i = 0; i < 4; ++i) P[j][i] = Q[j][i] = (Acc)0;

  const PhaseTab pt{lut, 2.f * (float)T, 1.f / (2.f * (float)T), 1.f / (float)T, 2 * T};

  using RingT = std::conditional_t<F32, f32x4, typename std::conditional_t<F32, Planes<BF_PLANES_FP16>, PT>::V4>;

  for (int k = 0; k <= K; ++k) {
    const float kf = (float)k;
    const Acc dk = (Acc)job.d[k];
    auto run = [&](auto nplc) {
      constexpr int NPL = decltype(nplc)::value;  // 1 for k = 0 (plane f - c0 only), else 4
      RingT ring[NT][NPL];
      static_for<0, NS>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int b = s & 1;
        const int ybase = Y0 - W + 16 * s;
        // ---- 1. modulate 16 rows into LDS buffer b
        constexpr int CW = F32 ? 4 : 8;  // pixels per thread chunk
        constexpr int CPR = LWU / CW;
        for (int c = tid; c < 16 * CPR; c += 256) {
          const int r = c / CPR, cc = c - r * CPR;
          const float* rowp = src + (size_t)fold(ybase + r, H) * sp;
          const int gx = X0 - W + CW * cc;
          float fv[CW];
#pragma unroll
          for (int e = 0; e < CW; ++e) fv[e] = rowp[fold(gx + e, Wd)];
          E vc[CW], vs[CW], vfc[CW], vfs[CW];
#pragma unroll
          for (int e = 0; e < CW; ++e) {
            const float v = fv[e] - c0;
            if constexpr (NPL == 4) {
              float cs, sn;
              phase<INTEGER>(kf, fv[e], pt, cs, sn);
              vc[e] = (E)cs;
              vs[e] = (E)sn;
              vfc[e] = (E)(v * cs);
              vfs[e] = (E)(v * sn);
            } else {
              vfc[e] = (E)v;
            }
          }
          if constexpr (NPL == 4) {
            __builtin_memcpy(&planes[b][0][r][CW * cc], vc, sizeof(vc));
            __builtin_memcpy(&planes[b][1][r][CW * cc], vs, sizeof(vs));
            __builtin_memcpy(&planes[b][3][r][CW * cc], vfs, sizeof(vfs));
          }
          __builtin_memcpy(&planes[b][2][r][CW * cc], vfc, sizeof(vfc));
        }
        __syncthreads();
        // ---- 2. row pass for this wave's strip
#pragma unroll
        for (int pi = 0; pi < NPL; ++pi) {
          const int p = (NPL == 1) ? 2 : pi;
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
          if constexpr (F32) {
#pragma unroll
            for (int s4 = 0; s4 < NBR; ++s4)
              if (s4 < nks4)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(planes[b][p][n16][16 * wave + 4 * s4 + g],
                                                            brow[s4], acc, 0, 0, 0);
            ring[s % NT][pi] = acc;
          } else {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
              typename PT::V8 a;
              __builtin_memcpy(&a, &planes[b][p][n16][16 * wave + 32 * ks + 8 * g], sizeof(a));
              acc = PT::mma(a, brow[ks], acc);
            }
            typename PT::V4 v;
            for (int i = 0; i < 4; ++i) v[i] = (E)acc[i];
            ring[s % NT][pi] = v;
          }
        }
        // ---- 3. column pass + 4. demodulate, once the window is complete
        if constexpr (s >= NT - 1) {
          constexpr int j = s - NT + 1;
          Acc fb[NPL][4];
#pragma unroll
          for (int pi = 0; pi < NPL; ++pi) {
            if constexpr (F32) {
              // One MFMA chain per 16-row window tile, chains summed in
              // float64: the column pass is the last smoothing step, so its
              // rounding is not averaged away, and its partial sums carry
              // |f - c0| up to T / 2; short chains keep them small.
              for (int i = 0; i < 4; ++i) fb[pi][i] = 0.0;
              static_for<0, NT>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ring[(j + t) % NT][pi][i], bcol32[t][i], acc, 0, 0, 0);
#pragma unroll
                for (int i = 0; i < 4; ++i) fb[pi][i] += (double)acc[i];
              });
            } else {
              f32x4 acc = {0.f, 0.f, 0.f, 0.f};
              static_for<0, KS>([&](auto kc) {
                constexpr int ks = decltype(kc)::value;
                typename PT::V4 lo = ring[(j + 2 * ks) % NT][pi];
                typename PT::V4 hi;
                if constexpr (2 * ks + 1 < NT) hi = ring[(j + 2 * ks + 1) % NT][pi];
                else hi = typename PT::V4{(E)0.f, (E)0.f, (E)0.f, (E)0.f};
                typename PT::V8 a = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
                acc = PT::mma(a, bcol16[ks], acc);
              });
#pragma unroll
              for (int i = 0; i < 4; ++i) fb[pi][i] = acc[i];
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if constexpr (NPL == 4) {
              float cs, sn;
              phase<INTEGER>(kf, fo[j][i], pt, cs, sn);
              const Acc dc = dk * (Acc)cs, ds = dk * (Acc)sn;
              P[j][i] = fma_acc(dc, fb[2][i], fma_acc(ds, fb[3][i], P[j][i]));
              Q[j][i] = fma_acc(dc, fb[0][i], fma_acc(ds, fb[1][i], Q[j][i]));
            } else {
              P[j][i] = fma_acc(dk, fb[0][i], P[j][i]);
              Q[j][i] += q0;
            }
          }
        }
      });
    };
    if (k == 0) run(std::integral_constant<int, 1>{});
    else run(std::integral_constant<int, 4>{});
    __syncthreads();
  }

  // ---- 5. divide and store
  float* __restrict__ dst = job.dst;
  for (int j = 0; j < NJ; ++j) {
    const int yy = Y0 + 16 * j + n16;
    if (yy >= H) continue;
    for (int i = 0; i < 4; ++i) {
      const int xx = x0 + 4 * g + i;
      if (xx < Wd) dst[(size_t)yy * job.dst_pitch + xx] = (float)(P[j][i] / Q[j][i] + (Acc)c0);
    }
  }
}

template <int PREC, int NT, int TH, bool INTEGER>
hipError_t launch_t(const JobDesc& job, hipStream_t stream) {
  dim3 grid((job.width + kTileCols - 1) / kTileCols, (job.height + TH - 1) / TH);
  const size_t lds = sizeof(float2) * 2 * (size_t)job.T;
  hipLaunchKernelGGL((fused_kernel<PREC, NT, TH, INTEGER>), grid, dim3(256), lds, stream, job);
  return hipGetLastError();
}

}  // namespace fused_detail

template <int PREC, int NT>
hipError_t launch_fused_nt(const JobDesc& job, int th, hipStream_t stream) {
  const bool integer = (job.flags & BF_FLAG_INTEGER_INPUT) != 0;
  if (th <= 32) return integer ? fused_detail::launch_t<PREC, NT, 32, true>(job, stream) : fused_detail::launch_t<PREC, NT, 32, false>(job, stream);
  return integer ? fused_detail::launch_t<PREC, NT, 64, true>(job, stream) : fused_detail::launch_t<PREC, NT, 64, false>(job, stream);
}

}  // namespace bf
