#pragma once
// Fused shiftable bilateral filter for gfx950 (one image per launch): the
// shared-plane kernel, used for fp32 planes and for non-integer images
// (16-bit planes on integer images use the barrier-free kernel of
// bf_wave_impl.h).
//
// Computes eq. (9) of the paper through Algorithm 1 in its real (cos/sin)
// form: with theta_k(j) = k w f(j), w = pi / T, and c0 = T / 2,
//   Q(i) = sum_k d_k [cos theta_k(i) (w * C_k)(i) + sin theta_k(i) (w * S_k)(i)]
//   with C_k = cos theta_k, S_k = sin theta_k, and P(i) the same sum with
//   C_k = (f - c0) cos theta_k, S_k = (f - c0) sin theta_k; the k = 0 term is
//   d_0 (w * (f - c0)) for P and d_0 sum(w) for Q, and the output is
//   P / Q + c0.  Summing the harmonics +k and -k of eq. (4) with
//   c_{+-k} = d_k / 2 gives exactly this real form (relation after eq. (6)).
//
// Work decomposition.  A workgroup of NW waves owns a (16 NW)-column x
// TH-row output tile; wave w owns the 16-column strip [X0 + 16w, +16).
// For integer gray levels the haloed image tile is staged once into LDS
// (borders folded there), and for each harmonic k the workgroup first
// tabulates, for every gray level f in 0..T, the modulation values
// (cos, sin, (f - c0) cos, (f - c0) sin)(k w f) and the demodulation phase;
// every later lookup is indexed by f, so no per-pixel phase arithmetic is
// left.  The workgroup then walks down the tile in 16-row steps:
//   1. modulate 16 input rows (all strips plus the halo) into LDS planes --
//      each input pixel is modulated once per step and shared by the waves;
//   2. row pass: one MFMA banded-Toeplitz product per 32 (16-bit) or 4
//      (fp32) input columns, with the Toeplitz weights held in registers;
//      the 16x16 result of each plane stays in registers (a ring of the last
//      NT row tiles);
//   3. column pass: once the ring spans 16 output rows plus the W-row halos,
//      a second Toeplitz product runs straight from the ring registers (the
//      MFMA output layout of the row pass is, up to a fixed permutation of the
//      contraction index that the weights absorb, the input layout of the
//      column pass), so row-filtered planes never touch LDS or HBM;
//   4. demodulate at the 16x16 output pixels and accumulate P, Q in
//      registers.
// Non-integer images take a general path that computes the phase per pixel
// (the integer part of k f through the cos/sin table of pi m / T, the
// fractional part by an explicit rotation).
#include <hip/hip_runtime.h>
#include <stdint.h>

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

// kRefineQ: denominators (unit-sum weights) below this are re-evaluated
// directly (see refine_pixels); the rounding error of the numerator and
// denominator sums divided by Q is the output error, and for Q down to w(0)
// that division amplifies it up to a few hundred times.
template <>
struct Planes<BF_PLANES_FP32> {
  using E = float;
  static constexpr float kRefineQ = 0.005f;
  static __device__ __forceinline__ float round(float x) { return x; }
};

// 16-bit formats.  E / V8 / V4 / mma / round: the modulated planes and the
// row-pass weights (the plane format).  RE / RV8 / RV4 / mma_col / round_col:
// the row-smoothed intermediate and the column-pass weights, which are
// float16 for both formats -- rounding that intermediate is the larger of
// bfloat16's two error sources, and its 8-bit mantissa alone keeps the
// result well away from half a gray level on the UHD workload.
struct RingF16 {
  using RE = _Float16;
  using RV8 = f16x8;
  using RV4 = f16x4;
  static __device__ __forceinline__ float round_col(float x) { return (float)(_Float16)x; }
  static __device__ __forceinline__ f32x4 mma_col(RV8 a, RV8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Planes<BF_PLANES_FP16> : RingF16 {
  static constexpr float kRefineQ = 0.02f;
  using E = _Float16;
  using V8 = f16x8;
  using V4 = f16x4;
  static __device__ __forceinline__ float round(float x) { return (float)(_Float16)x; }
  static __device__ __forceinline__ uint32_t bits(float x) {
    return __builtin_bit_cast(uint16_t, (_Float16)x);
  }
  static __device__ __forceinline__ f32x4 mma(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Planes<BF_PLANES_BF16> : RingF16 {
  static constexpr float kRefineQ = 0.05f;
  using E = __bf16;
  using V8 = b16x8;
  using V4 = b16x4;
  static __device__ __forceinline__ float round(float x) { return (float)(__bf16)x; }
  static __device__ __forceinline__ uint32_t bits(float x) {
    return __builtin_bit_cast(uint16_t, (__bf16)x);
  }
  static __device__ __forceinline__ f32x4 mma(V8 a, V8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// the 16-bit traits of a format (fp32 maps to fp16; only used in branches
// that fp32 planes never take)
template <int PREC>
using PlanesOr16 = Planes<PREC == BF_PLANES_FP32 ? BF_PLANES_FP16 : PREC>;

// Tile geometry shared by the kernel and its launcher.
template <int PREC, int NT>
struct Geo {
  static constexpr bool F32 = (PREC == BF_PLANES_FP32);
  static constexpr int NW = F32 ? 4 : 8;                  // waves per workgroup
  static constexpr int THREADS = 64 * NW;
  static constexpr int COLS = 16 * NW;                    // output columns per workgroup
  static constexpr int KS = (NT + 1) / 2;                 // 32-column contraction steps
  static constexpr int LWU = 16 * (NW - 1) + 32 * KS;     // staged input columns
  static constexpr int LW = F32 ? LWU + 4 : LWU + 8;      // padded plane row (elements)
  static constexpr int FW = LWU + 8;                      // padded image-tile row (u16)
};

constexpr int kTabBytes = 16;  // one table entry per gray level
constexpr size_t kLdsLimit = 160 * 1024;

template <int PREC>
constexpr int kThreadsFor = (PREC == BF_PLANES_FP32) ? 256 : 512;

// static LDS of one instantiation, and whether its staged image tile fits
template <int PREC, int NT, int TH, bool INTEGER>
struct Lds {
  using G = Geo<PREC, NT>;
  // FP32 planes on integer images gather their operands per lane and keep no
  // planes in LDS
  static constexpr size_t planes = (G::F32 && INTEGER) ? 0 : 2ull * 4 * 16 * G::LW * (G::F32 ? 4 : 2);
  static constexpr size_t tile = INTEGER ? 2ull * 16 * (TH / 16 + NT - 1) * G::FW : 16;
  static constexpr size_t total = planes + tile + 4 * (2 * BF_MAX_W + 1) + 64;
  // a staged variant must leave room for at least the T = 255 tables
  static constexpr bool fits = total + kTabBytes * 256 + 8 * 510 <= kLdsLimit;
};

inline size_t dynamic_lds(int T, int F) { return (size_t)kTabBytes * (F + 1) + sizeof(float2) * 2 * (size_t)T; }

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

// Stage a rows x cols block of the image starting at (y0, x0), folded at the
// borders: element (r, c) is read and handed to put(r, c, v).  Each thread
// issues a batch of independent global reads before it uses any of them, so
// their latencies overlap (one read and wait per element would serialise a
// full memory round trip per element).  Blocks whose columns lie inside the
// image, start 16-byte aligned and span a multiple of 4 columns are read as
// float4: a thread keeps one column quad and steps down the rows, so that its
// addresses need no per-element division; others element by element with the
// border fold.
constexpr int kStageBatch = 16;
constexpr int kStageBatch4 = 24;
typedef float f4v_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bool stage_vectorizable(const float* src, int pitch, int cols, int x0, int Wd) {
  return x0 >= 0 && x0 + cols <= Wd && (cols & 3) == 0 && (pitch & 3) == 0 &&
         ((reinterpret_cast<uintptr_t>(src) + 4 * (uintptr_t)x0) & 15) == 0;
}

template <int NTHREADS, typename Put>
__device__ __forceinline__ void stage_tile(const float* src, int pitch, int rows, int cols, int y0, int x0, int H,
                                           int Wd, Put put) {
  const __attribute__((address_space(1))) float* g = (const __attribute__((address_space(1))) float*)src;
  if (stage_vectorizable(src, pitch, cols, x0, Wd) && (cols >> 2) <= NTHREADS) {
    const int q4 = cols >> 2, rstep = NTHREADS / q4;
    const int r0 = (int)threadIdx.x / q4, c = 4 * ((int)threadIdx.x - r0 * q4);
    if (r0 >= rstep) return;  // threads beyond the last whole row of quads
    for (int rb = r0; rb < rows; rb += kStageBatch4 * rstep) {
      f4v_t v[kStageBatch4];
#pragma unroll
      for (int b = 0; b < kStageBatch4; ++b) {
        const int r = rb + b * rstep;
        v[b] = r < rows ? *reinterpret_cast<const __attribute__((address_space(1))) f4v_t*>(
                              g + (size_t)fold(y0 + r, H) * pitch + x0 + c)
                        : f4v_t{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int b = 0; b < kStageBatch4; ++b) {
        const int r = rb + b * rstep;
        if (r < rows) {
          put(r, c, v[b].x);
          put(r, c + 1, v[b].y);
          put(r, c + 2, v[b].z);
          put(r, c + 3, v[b].w);
        }
      }
    }
    return;
  }
  // element idx = r * cols + c; a thread's elements are NTHREADS apart
  const int dr = NTHREADS / cols, dc = NTHREADS - dr * cols;
  int r = (int)threadIdx.x / cols, c = (int)threadIdx.x - r * cols;
  while (r < rows) {
    float v[kStageBatch];
    int rc[kStageBatch];
#pragma unroll
    for (int b = 0; b < kStageBatch; ++b) {
      rc[b] = (r << 16) | c;
      v[b] = r < rows ? g[(size_t)fold(y0 + r, H) * pitch + fold(x0 + c, Wd)] : 0.f;
      r += dr;
      c += dc;
      if (c >= cols) {
        c -= cols;
        ++r;
      }
    }
#pragma unroll
    for (int b = 0; b < kStageBatch; ++b)
      if ((rc[b] >> 16) < rows) put(rc[b] >> 16, rc[b] & 0xffff, v[b]);
  }
}

// Read-ahead of one tile's block (ROWS x COLS) into registers: the float4 path
// of stage_tile split into issue() (the reads start) and commit() (the values
// go to put(r, c, v)), so that a persistent workgroup can start the reads of
// its next tile before it finishes the current one.
template <int NTHREADS, int ROWS, int COLS>
struct TileReadAhead {
  static constexpr int Q4 = COLS / 4, RSTEP = NTHREADS / Q4, NB = (ROWS + RSTEP - 1) / RSTEP;
  static_assert(COLS % 4 == 0 && Q4 <= NTHREADS, "a row of quads per pass");
  f4v_t v[NB];
  bool valid;
  __device__ static bool eligible(const float* src, int pitch, int x0, int Wd) {
    return stage_vectorizable(src, pitch, COLS, x0, Wd);
  }
  __device__ void issue(const float* src, int pitch, int y0, int x0, int H) {
    const __attribute__((address_space(1))) float* g = (const __attribute__((address_space(1))) float*)src;
    const int r0 = (int)threadIdx.x / Q4, c = 4 * ((int)threadIdx.x - r0 * Q4);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int r = r0 + b * RSTEP;
      v[b] = (r0 < RSTEP && r < ROWS) ? *reinterpret_cast<const __attribute__((address_space(1))) f4v_t*>(
                                            g + (size_t)fold(y0 + r, H) * pitch + x0 + c)
                                      : f4v_t{0.f, 0.f, 0.f, 0.f};
    }
  }
  __device__ void clear() {
#pragma unroll
    for (int b = 0; b < NB; ++b) v[b] = f4v_t{0.f, 0.f, 0.f, 0.f};
  }
  template <typename Put>
  __device__ void commit(Put put) const {
    const int r0 = (int)threadIdx.x / Q4, c = 4 * ((int)threadIdx.x - r0 * Q4);
    if (r0 >= RSTEP) return;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int r = r0 + b * RSTEP;
      if (r < ROWS) {
        put(r, c, v[b].x);
        put(r, c + 1, v[b].y);
        put(r, c + 2, v[b].z);
        put(r, c + 3, v[b].w);
      }
    }
  }
};

__device__ __forceinline__ float fma_acc(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_acc(double a, double b, double c) { return fma(a, b, c); }

// m -> (cos, sin)(pi m / T), m = 0..2T-1, for the general (non-integer) path
struct PhaseTab {
  const float2* lut;
  float two_t, inv_two_t, inv_t;
  int n_lut;  // 2T
};

__device__ __forceinline__ float reduce_2t(float p, const PhaseTab& pt) {
  const float q = floorf(p * pt.inv_two_t);
  float m = fmaf(-pt.two_t, q, p);
  m = (m >= pt.two_t) ? m - pt.two_t : m;
  return (m < 0.f) ? m + pt.two_t : m;
}

// cos and sin of k w f, any real f: k f = k floor(f) + k frac(f); the integer
// part indexes the table exactly, the remaining fraction r in [0, 1) is
// applied as a rotation by pi r / T
__device__ __forceinline__ void phase_general(float kf, float f, const PhaseTab& pt, float& c, float& s) {
  const float fi = floorf(f);
  const float pf = kf * (f - fi);
  const float n2 = floorf(pf);
  const float r = pf - n2;
  const float m = reduce_2t(fmaf(kf, fi, n2), pt);
  const float2 v = pt.lut[min(max((int)m, 0), pt.n_lut - 1)];  // clamp: non-finite input
  float sr, cr;
  sincospif(r * pt.inv_t, &sr, &cr);
  c = v.x * cr - v.y * sr;
  s = v.y * cr + v.x * sr;
}

// ---- direct re-evaluation of ill-conditioned pixels -----------------------
// The output is P / Q + c0, and rounding errors in P and Q (16-bit planes
// and intermediates, or fp32 sums) reach the output divided by Q.  With a
// unit-sum spatial kernel Q can be as small as the centre weight w(0) at a
// pixel whose window holds no other gray level within the range kernel's
// reach, so there the Fourier-plane sums are re-evaluated directly: eq. (9)
// written out over the (2W+1)^2 window with phi_K tabulated on the integer
// differences 0..F, in float64.  These pixels are rare (a few in 10^4 on
// natural-looking images) and the kernels find them from their own Q.

// phi_K(t) = sum_k d_k cos(k w t), t = 0..F, into phi (float64, LDS); lut
// holds cos/sin(pi m / T), m = 0..2T-1.  Called by every thread.
__device__ __forceinline__ void build_phi_table(const JobDesc& job, const float2* lut, double* phi, int nthreads) {
  const int T2 = 2 * job.T;
  for (int t = threadIdx.x; t <= job.F; t += nthreads) {
    double acc = job.d[0];
    int m = 0;
    for (int k = 1; k <= job.K; ++k) {
      m += t;
      m = m >= T2 ? m % T2 : m;  // (k t) mod 2T
      acc = fma(job.d[k], (double)lut[m].x, acc);
    }
    phi[t] = acc;
  }
}

// Bit 4 j + i of the returned mask: output (j, i) of this lane lies inside
// the image and has !(Q >= tau) (NaN included).
template <int NJ, class Acc>
__device__ __forceinline__ unsigned long long refine_flags(const Acc (&Q)[NJ][4], const JobDesc& job, int Y0, int x0,
                                                           float tau) {
  const int lane = threadIdx.x & 63;
  unsigned long long fl = 0;
#pragma unroll
  for (int j = 0; j < NJ; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int yy = Y0 + 16 * j + (lane & 15), xx = x0 + 4 * (lane >> 4) + i;
      if (yy < job.height && xx < job.width && !(Q[j][i] >= (Acc)tau)) fl |= 1ull << (4 * j + i);
    }
  return fl;
}

// Eq. (9) evaluated directly at one output pixel by the whole wave, written
// to dst: the pixel sits at (r, c) from the output tile's origin (X0, Y0),
// at staged-tile row W + r and column corg + c.  Lane l takes window
// columns l, l + 64, ...; the rows of a column are independent loads (so
// several are in flight), summed in float64, and a butterfly sums the lanes.
template <class Gray>
__device__ __forceinline__ void refine_pixel(int r, int c, const JobDesc& job, int X0, int Y0, int corg,
                                             const float* w1s, const double* phi, Gray gray) {
  const int lane = threadIdx.x & 63;
  const int W = job.W;
  const double c0 = (double)job.c0;
  const int tr = W + r, tc = corg + c;
  const int fi = gray(tr, tc);
  double p = 0.0, q = 0.0;
  for (int dx = lane; dx <= 2 * W; dx += 64) {
    double pc = 0.0, qc = 0.0;
#pragma unroll 4
    for (int dy = 0; dy <= 2 * W; ++dy) {
      const int fj = gray(tr - W + dy, tc - W + dx);
      const double wp = (double)w1s[dy] * phi[fj >= fi ? fj - fi : fi - fj];
      qc += wp;
      pc = fma(wp, (double)fj - c0, pc);
    }
    const double wx = (double)w1s[dx];
    p = fma(wx, pc, p);
    q = fma(wx, qc, q);
  }
  for (int o = 32; o >= 1; o >>= 1) {
    p += __shfl_xor(p, o);
    q += __shfl_xor(q, o);
  }
  if (lane == 0) job.dst[(size_t)(Y0 + r) * job.dst_pitch + X0 + c] = (float)(p / q + c0);
}

// The same evaluation by one thread alone (the fallback for a pixel that
// does not fit the shared list).
template <class Gray>
__device__ __forceinline__ void refine_pixel_alone(int r, int c, const JobDesc& job, int X0, int Y0, int corg,
                                                   const float* w1s, const double* phi, Gray gray) {
  const int W = job.W;
  const double c0 = (double)job.c0;
  const int tr = W + r, tc = corg + c;
  const int fi = gray(tr, tc);
  double p = 0.0, q = 0.0;
  for (int dy = 0; dy <= 2 * W; ++dy) {
    double pr = 0.0, qr = 0.0;
    for (int dx = 0; dx <= 2 * W; ++dx) {
      const int fj = gray(tr - W + dy, tc - W + dx);
      const double wp = (double)w1s[dx] * phi[fj >= fi ? fj - fi : fi - fj];
      qr += wp;
      pr = fma(wp, (double)fj - c0, pr);
    }
    p = fma((double)w1s[dy], pr, p);
    q = fma((double)w1s[dy], qr, q);
  }
  job.dst[(size_t)(Y0 + r) * job.dst_pitch + X0 + c] = (float)(p / q + c0);
}

// Re-evaluates the flagged outputs of a workgroup's tile after the tile's
// outputs have been stored.  Called by every thread with `any` (whether it
// holds flagged outputs) and `each(emit)`, which calls emit(r, c) for each of
// them, (r, c) counted from the tile's output origin (X0, Y0); gray(r, c)
// reads staged-tile coordinates, where output (r, c) sits at row W + r and
// column corg + c.  The flagged pixels are pooled in an LDS list so that all
// waves share them; `scratch` (LDS free at this point, 16-byte aligned)
// holds phi_K on 0..F and the list; a pixel beyond the list's room is done
// by its own thread alone.
template <class Each, class Gray>
__device__ __forceinline__ void refine_pooled(bool any, Each each, const JobDesc& job, int X0, int Y0, int corg,
                                              const float* w1s, const float2* lut, unsigned char* scratch,
                                              size_t scratch_bytes, int nthreads, Gray gray) {
  // also the barrier after which every wave is done with the tables
  if (!__syncthreads_or(any)) return;
  const int tid = threadIdx.x, wave = tid >> 6, nwaves = nthreads >> 6;
  double* phi = reinterpret_cast<double*>(scratch);
  const size_t phi_bytes = (8 * (size_t)(job.F + 1) + 15) & ~(size_t)15;
  int* cnt = reinterpret_cast<int*>(scratch + phi_bytes);
  uint32_t* lst = reinterpret_cast<uint32_t*>(scratch + phi_bytes + 16);
  const int cap = scratch_bytes > phi_bytes + 16 ? (int)((scratch_bytes - phi_bytes - 16) / 4) : 0;
  build_phi_table(job, lut, phi, nthreads);
  if (tid == 0) *cnt = 0;
  __syncthreads();
  each([&](int r, int c) {
    const int idx = atomicAdd(cnt, 1);
    if (idx < cap) lst[idx] = (uint32_t)r | ((uint32_t)c << 16);
    else refine_pixel_alone(r, c, job, X0, Y0, corg, w1s, phi, gray);
  });
  __syncthreads();
  const int n = min(*cnt, cap);
  for (int e = wave; e < n; e += nwaves) {
    const uint32_t v = lst[e];
    refine_pixel((int)(v & 0xffffu), (int)(v >> 16), job, X0, Y0, corg, w1s, phi, gray);
  }
}

// refine_pooled for the MFMA kernels' layout: bit 4 j + i of a lane's mask
// (refine_flags) is output (16 j + n16, 16 w + 4 g + i) of lane (g, n16) of
// wave w.
template <int NJ, class Gray>
__device__ __forceinline__ void refine_tile(unsigned long long fl, const JobDesc& job, int X0, int Y0, int corg,
                                            const float* w1s, const float2* lut, unsigned char* scratch,
                                            size_t scratch_bytes, int nthreads, Gray gray) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  refine_pooled(fl != 0, [&](auto&& emit) {
    for (unsigned long long m = fl; m; m &= m - 1) {
      const int b = __ffsll((long long)m) - 1;
      emit(16 * (b >> 2) + (lane & 15), 16 * wave + 4 * (lane >> 4) + (b & 3));
    }
  }, job, X0, Y0, corg, w1s, lut, scratch, scratch_bytes, nthreads, gray);
}

// One output tile (COLS x TH at X0, Y0) of one image, all harmonics.  smem
// holds the plane buffers, the staged tile and the spatial profile (layout of
// Lds<>); tab has room for (T+1) 16-byte entries; lut holds cos/sin(pi m / T),
// rebuilt here when build_lut is set.  Every thread of the workgroup must call
// it (it contains barriers).
template <int PREC, int NT, int TH, bool INTEGER_REQ>
__device__ __forceinline__ void fused_tile(const JobDesc& job, int X0, int Y0, unsigned char* smem,
                                           unsigned char* tab, float2* lut, bool build_lut) {
  constexpr bool INTEGER = INTEGER_REQ && Lds<PREC, NT, TH, true>::fits;
  using G = Geo<PREC, NT>;
  // FP32 planes on integer images: each lane gathers its row-pass operands
  // (all four plane values of a pixel, one 16-byte table entry) straight
  // from the table, so no planes go through LDS and no barrier is needed
  // between the 16-row steps
  constexpr bool DIRECT = G::F32 && INTEGER;
  using PT = Planes<PREC>;
  using E = typename PT::E;
  constexpr bool F32 = G::F32;
  constexpr int NTHR = G::THREADS, KS = G::KS, LWU = G::LWU, LW = G::LW, FW = G::FW;
  constexpr int NJ = TH / 16;            // output row tiles per workgroup
  constexpr int NS = NJ + NT - 1;        // 16-row steps per harmonic
  constexpr int FROWS = 16 * NS;         // staged image rows

  using L = Lds<PREC, NT, TH, INTEGER>;
  auto planes = reinterpret_cast<E(*)[4][16][LW]>(smem);
  // image tile, stored as f * kTabBytes (byte offset of gray level f in the table)
  auto ftile = reinterpret_cast<uint16_t(*)[INTEGER ? FW : 8]>(smem + L::planes);
  float* w1s = reinterpret_cast<float*>(smem + L::planes + L::tile);

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, n16 = lane & 15;
  const int x0 = X0 + 16 * wave;
  const int W = job.W, T = job.T, K = job.K;
  const int Wal = (W + 7) & ~7;          // column origin of the staged tile: X0 - Wal
  const int H = job.height, Wd = job.width;
  const float* __restrict__ src = job.src;
  const int sp = job.src_pitch;
  const float c0 = job.c0;
  for (int m = tid; m < (build_lut ? 2 * T : 0); m += NTHR) {
    double s, c;
    sincospi((double)m / (double)T, &s, &c);
    lut[m] = make_float2((float)c, (float)s);
  }
  for (int t = tid; t <= 2 * W; t += NTHR) w1s[t] = job.w1[t];
  if constexpr (INTEGER) {
    const float Fm = (float)job.F;
    stage_tile<NTHR>(src, sp, FROWS, LWU, Y0 - W, X0 - Wal, H, Wd, [&](int r, int c, float v) {
      v = fminf(fmaxf(v, 0.f), Fm);  // NaN -> 0; the flag promises integers in [0, F]
      ftile[r][c] = (uint16_t)((int)v * kTabBytes);
    });
  }
  __syncthreads();

  auto wq = [&](int dd) -> float { return (dd >= -W && dd <= W) ? PT::round(w1s[dd + W]) : 0.f; };
  // column-pass weights: rounded like the row-smoothed intermediate (float16)
  // for 16-bit planes, unrounded for fp32
  auto wqc = [&](int dd) -> float {
    if constexpr (F32) return wq(dd);
    else return (dd >= -W && dd <= W) ? PlanesOr16<PREC>::round_col(w1s[dd + W]) : 0.f;
  };

  // Toeplitz operands.  Row pass: B[k][n] = w(input col - output col), the
  // input col of contraction slot k counted from x0 - Wal.  Column pass: the
  // contraction slot (lane group g, element e) holds row 4g + (e & 3) of ring
  // tile 2ks + (e >> 2) (16-bit) or row 4g + i of ring tile t (fp32), rows
  // counted from the output row - W.
  using BrowT = std::conditional_t<F32, float, typename std::conditional_t<F32, Planes<BF_PLANES_FP16>, PT>::V8>;
  constexpr int NBR = F32 ? 8 * KS : KS;
  using BcolT = std::conditional_t<F32, float, typename std::conditional_t<F32, Planes<BF_PLANES_FP16>, PT>::RV8>;
  BrowT brow[NBR];
  float bcol32[F32 ? NT : 1][4];
  BcolT bcol16[F32 ? 1 : KS];
  if constexpr (F32) {
    for (int s4 = 0; s4 < NBR; ++s4) brow[s4] = wq(4 * s4 + g - Wal - n16);
    for (int t = 0; t < NT; ++t)
      for (int i = 0; i < 4; ++i) bcol32[t][i] = wq(16 * t + 4 * g + i - W - n16);
  } else {
    for (int ks = 0; ks < KS; ++ks)
      for (int e = 0; e < 8; ++e) {
        brow[ks][e] = (E)wq(32 * ks + 8 * g + e - Wal - n16);
        bcol16[ks][e] = (typename PlanesOr16<PREC>::RE)wqc(16 * (2 * ks + (e >> 2)) + 4 * g + (e & 3) - W - n16);
      }
  }
  // fp32 planes accumulate P and Q in float64 (see the column pass below);
  // 16-bit planes are limited by their own rounding and accumulate in float32
  using Acc = std::conditional_t<F32, double, float>;
  // k = 0: Q gains d_0 times the smoothing of the ones-plane, i.e. the
  // product of the row and column weight sums
  double wsum_r = 0.0, wsum_c = 0.0;
  for (int t = -W; t <= W; ++t) {
    wsum_r += (double)wq(t);
    wsum_c += (double)wqc(t);
  }
  const Acc q0 = (Acc)(job.d[0] * wsum_r * wsum_c);

  // general path: gray levels at this lane's output pixels (row Y0 + 16 j + n16, cols x0 + 4 g + i)
  float fo[INTEGER ? 1 : NJ][4];
  if constexpr (!INTEGER) {
    for (int j = 0; j < NJ; ++j)
      for (int i = 0; i < 4; ++i) {
        const int yy = min(Y0 + 16 * j + n16, H - 1), xx = min(x0 + 4 * g + i, Wd - 1);
        fo[j][i] = src[(size_t)yy * sp + xx];
      }
  }
  Acc P[NJ][4], Q[NJ][4];
  for (int j = 0; j < NJ; ++j)
    for (int i = 0; i < 4; ++i) P[j][i] = Q[j][i] = (Acc)0;

  const PhaseTab pt{lut, 2.f * (float)T, 1.f / (2.f * (float)T), 1.f / (float)T, 2 * T};
  const float two_t = 2.f * (float)T, inv_two_t = 1.f / (2.f * (float)T);

  using RingT = std::conditional_t<F32, f32x4, typename std::conditional_t<F32, Planes<BF_PLANES_FP16>, PT>::RV4>;

  for (int k = 0; k <= K; ++k) {
    const float kf = (float)k;
    const Acc dk = (Acc)job.d[k];
    __syncthreads();  // every wave is done with harmonic k - 1 (table and planes)
    if constexpr (INTEGER) {
      // per-harmonic table, entry f: fp32 (c, s, (f-c0) c, (f-c0) s) for fp32
      // planes; for 16-bit planes (d_k c, d_k s) in fp32 for the demodulation
      // and (c, s, (f-c0) c, (f-c0) s) rounded to the plane format
      for (int f = tid; f <= job.F; f += NTHR) {
        const float m = reduce_2t((float)k * (float)f, pt);
        const float2 cs = lut[min(max((int)m, 0), 2 * T - 1)];
        const float v = (float)f - c0;
        unsigned char* ent = tab + (size_t)kTabBytes * f;
        if constexpr (F32) {
          *reinterpret_cast<float4*>(ent) = make_float4(cs.x, cs.y, v * cs.x, v * cs.y);
        } else {
          const float dkf = (float)job.d[k];
          const uint32_t w0 = PT::bits(cs.x) | (PT::bits(cs.y) << 16);
          const uint32_t w1 = PT::bits(v * cs.x) | (PT::bits(v * cs.y) << 16);
          *reinterpret_cast<uint4*>(ent) =
              make_uint4(__float_as_uint(dkf * cs.x), __float_as_uint(dkf * cs.y), w0, w1);
        }
      }
      __syncthreads();
    }
    auto run = [&](auto nplc) {
      constexpr int NPL = decltype(nplc)::value;  // 1 for k = 0 (plane f - c0 only), else 4
      RingT ring[NT][NPL];
      // ---- 1. modulate rows [16 sm, 16 sm + 16) of the tile into LDS buffer
      // sm & 1, one 8-pixel chunk per thread and pass; branch-free (lanes past
      // the last chunk repeat it, writing the same values), so that it can
      // interleave with the MFMAs of the step it overlaps
      auto modulate = [&](auto smc) {
        if constexpr (DIRECT) return;  // no LDS planes (the rest is never run)
        constexpr int s = decltype(smc)::value;
        constexpr int b = s & 1;
        constexpr int CPR = LWU / 8;  // 8-pixel chunks per row
        constexpr int NCH = 16 * CPR;
#pragma unroll
        for (int it = 0; it < (NCH + NTHR - 1) / NTHR; ++it) {
          const int c = min(tid + it * NTHR, NCH - 1);
          const int r = c / CPR, cc = c - r * CPR;
          if constexpr (INTEGER) {
            const uint4 fq = *reinterpret_cast<const uint4*>(&ftile[16 * s + r][8 * cc]);
            const uint32_t fw[4] = {fq.x, fq.y, fq.z, fq.w};
            if constexpr (F32) {
              float pc[8], ps[8], pfc[8], pfs[8];
#pragma unroll
              for (int e = 0; e < 8; ++e) {
                const uint32_t off = (e & 1) ? (fw[e >> 1] >> 16) : (fw[e >> 1] & 0xffffu);
                const float4 t = *reinterpret_cast<const float4*>(tab + off);
                pc[e] = t.x; ps[e] = t.y; pfc[e] = t.z; pfs[e] = t.w;
              }
              if constexpr (NPL == 4) {
                __builtin_memcpy(&planes[b][0][r][8 * cc], pc, sizeof(pc));
                __builtin_memcpy(&planes[b][1][r][8 * cc], ps, sizeof(ps));
                __builtin_memcpy(&planes[b][3][r][8 * cc], pfs, sizeof(pfs));
              }
              __builtin_memcpy(&planes[b][2][r][8 * cc], pfc, sizeof(pfc));
            } else {
              uint32_t pc[4], ps[4], pfc[4], pfs[4];
#pragma unroll
              for (int h = 0; h < 4; ++h) {  // pixels 2h, 2h + 1
                const uint2 ta = *reinterpret_cast<const uint2*>(tab + (fw[h] & 0xffffu) + 8);
                const uint2 tb = *reinterpret_cast<const uint2*>(tab + (fw[h] >> 16) + 8);
                pc[h] = (ta.x & 0xffffu) | (tb.x << 16);
                ps[h] = (ta.x >> 16) | (tb.x & 0xffff0000u);
                pfc[h] = (ta.y & 0xffffu) | (tb.y << 16);
                pfs[h] = (ta.y >> 16) | (tb.y & 0xffff0000u);
              }
              if constexpr (NPL == 4) {
                __builtin_memcpy(&planes[b][0][r][8 * cc], pc, sizeof(pc));
                __builtin_memcpy(&planes[b][1][r][8 * cc], ps, sizeof(ps));
                __builtin_memcpy(&planes[b][3][r][8 * cc], pfs, sizeof(pfs));
              }
              __builtin_memcpy(&planes[b][2][r][8 * cc], pfc, sizeof(pfc));
            }
          } else {
            const float* rowp = src + (size_t)fold(Y0 - W + 16 * s + r, H) * sp;
            const int gx = X0 - Wal + 8 * cc;
            E vc[8], vs[8], vfc[8], vfs[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const float fv = rowp[fold(gx + e, Wd)];
              const float v = fv - c0;
              if constexpr (NPL == 4) {
                float cs, sn;
                phase_general(kf, fv, pt, cs, sn);
                vc[e] = (E)cs;
                vs[e] = (E)sn;
                vfc[e] = (E)(v * cs);
                vfs[e] = (E)(v * sn);
              } else {
                vfc[e] = (E)v;
              }
            }
            if constexpr (NPL == 4) {
              __builtin_memcpy(&planes[b][0][r][8 * cc], vc, sizeof(vc));
              __builtin_memcpy(&planes[b][1][r][8 * cc], vs, sizeof(vs));
              __builtin_memcpy(&planes[b][3][r][8 * cc], vfs, sizeof(vfs));
            }
            __builtin_memcpy(&planes[b][2][r][8 * cc], vfc, sizeof(vfc));
          }
        }
      };
      modulate(std::integral_constant<int, 0>{});
      static_for<0, NS>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int b = s & 1;
        // buffer b complete; every wave is done with step s - 1, so buffer
        // b ^ 1 (read by its row pass) may be overwritten below
        if constexpr (!DIRECT) __syncthreads();
        // ---- 2. row pass for this wave's strip
        float4 tv[DIRECT ? NBR : 1];
        if constexpr (DIRECT) {
#pragma unroll
          for (int s4 = 0; s4 < NBR; ++s4)
            tv[s4] = *reinterpret_cast<const float4*>(tab + ftile[16 * s + n16][16 * wave + 4 * s4 + g]);
        }
#pragma unroll
        for (int pi = 0; pi < NPL; ++pi) {
          const int p = (NPL == 1) ? 2 : pi;
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
          if constexpr (F32) {
            // every contraction step of the class, in one branch-free block:
            // the steps outside this window's column span have zero weights
            // and add exact zeros, and without branches the operand reads
            // run ahead of the MFMA chain
            float av[NBR];
#pragma unroll
            for (int s4 = 0; s4 < NBR; ++s4) {
              if constexpr (DIRECT)
                av[s4] = p == 0 ? tv[s4].x : p == 1 ? tv[s4].y : p == 2 ? tv[s4].z : tv[s4].w;
              else
                av[s4] = planes[b][p][n16][16 * wave + 4 * s4 + g];
            }
#pragma unroll
            for (int s4 = 0; s4 < NBR; ++s4) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[s4], brow[s4], acc, 0, 0, 0);
            ring[s % NT][pi] = acc;
          } else {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
              typename PT::V8 a;
              __builtin_memcpy(&a, &planes[b][p][n16][16 * wave + 32 * ks + 8 * g], sizeof(a));
              acc = PT::mma(a, brow[ks], acc);
            }
            RingT v;
            for (int i = 0; i < 4; ++i) v[i] = (typename PlanesOr16<PREC>::RE)acc[i];
            ring[s % NT][pi] = v;
          }
        }
        // modulation of the next step into the other buffer, overlapping
        // this step's matrix work
        if constexpr (s + 1 < NS) modulate(std::integral_constant<int, s + 1>{});
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
                using R16 = PlanesOr16<PREC>;
                typename R16::RV4 lo = ring[(j + 2 * ks) % NT][pi];
                typename R16::RV4 hi;
                if constexpr (2 * ks + 1 < NT) hi = ring[(j + 2 * ks + 1) % NT][pi];
                else hi = typename R16::RV4{(typename R16::RE)0.f, (typename R16::RE)0.f, (typename R16::RE)0.f,
                                            (typename R16::RE)0.f};
                typename R16::RV8 a = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
                acc = R16::mma_col(a, bcol16[ks], acc);
              });
#pragma unroll
              for (int i = 0; i < 4; ++i) fb[pi][i] = acc[i];
            }
          }
          // demodulation phase at pixels (Y0 + 16 j + n16, x0 + 4 g + i)
          Acc dcs[4], dsn[4];
          if constexpr (NPL == 4) {
            if constexpr (INTEGER) {
              const uint2 fq = *reinterpret_cast<const uint2*>(&ftile[W + 16 * j + n16][Wal + 16 * wave + 4 * g]);
              const uint32_t off[4] = {fq.x & 0xffffu, fq.x >> 16, fq.y & 0xffffu, fq.y >> 16};
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const float2 t = *reinterpret_cast<const float2*>(tab + off[i]);
                if constexpr (F32) {
                  dcs[i] = dk * (Acc)t.x;
                  dsn[i] = dk * (Acc)t.y;
                } else {
                  dcs[i] = t.x;  // the 16-bit table already holds d_k cos, d_k sin
                  dsn[i] = t.y;
                }
              }
            } else {
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                float cs, sn;
                phase_general(kf, fo[j][i], pt, cs, sn);
                dcs[i] = dk * (Acc)cs;
                dsn[i] = dk * (Acc)sn;
              }
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            if constexpr (NPL == 4) {
              P[j][i] = fma_acc(dcs[i], fb[2][i], fma_acc(dsn[i], fb[3][i], P[j][i]));
              Q[j][i] = fma_acc(dcs[i], fb[0][i], fma_acc(dsn[i], fb[1][i], Q[j][i]));
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
  }

  // ---- 5. divide and store; then re-evaluate the ill-conditioned pixels
  // of integer images directly (see refine_pixels)
  float* __restrict__ dst = job.dst;
  for (int j = 0; j < NJ; ++j) {
    const int yy = Y0 + 16 * j + n16;
    if (yy >= H) continue;
    for (int i = 0; i < 4; ++i) {
      const int xx = x0 + 4 * g + i;
      if (xx < Wd) dst[(size_t)yy * job.dst_pitch + xx] = (float)(P[j][i] / Q[j][i] + (Acc)c0);
    }
  }
  if constexpr (INTEGER) {
    const unsigned long long fl = refine_flags<NJ>(Q, job, Y0, x0, PT::kRefineQ);
    refine_tile<NJ>(fl, job, X0, Y0, Wal, w1s, lut, tab, (size_t)kTabBytes * (job.F + 1), NTHR,
                    [&](int r, int c) { return (int)ftile[r][c] / kTabBytes; });
  }
  (void)two_t;
  (void)inv_two_t;
  __syncthreads();  // the LDS of this tile may be reused by the caller
}

template <int PREC, int NT, int TH, bool INTEGER>
__global__ void __launch_bounds__(kThreadsFor<PREC>) fused_kernel(const JobDesc job) {
  constexpr bool staged = INTEGER && Lds<PREC, NT, TH, true>::fits;
  __shared__ __attribute__((aligned(16))) unsigned char smem[Lds<PREC, NT, TH, staged>::total];
  // dynamic: per-harmonic table [(T+1) x 16 B], then cos/sin(pi m / T) [2T x 8 B]
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  fused_tile<PREC, NT, TH, INTEGER>(job, blockIdx.x * Geo<PREC, NT>::COLS, blockIdx.y * TH, smem, dyn,
                                    reinterpret_cast<float2*>(dyn + (size_t)kTabBytes * (job.F + 1)), true);
}

// Persistent form: workgroup b processes items b, b + gridDim.x, ... of a
// cost-ordered list; item = (job index, tile x0, tile y0, -).  Dynamic LDS:
// cos/sin table for T_max first, then the per-harmonic table.
template <int PREC, int NT, int TH, bool INTEGER>
__global__ void __launch_bounds__(kThreadsFor<PREC>) fused_batched_kernel(const JobDesc* __restrict__ jobs,
                                                                        const int4* __restrict__ items,
                                                                        int n_items, int t_max) {
  constexpr bool staged = INTEGER && Lds<PREC, NT, TH, true>::fits;
  __shared__ __attribute__((aligned(16))) unsigned char smem[Lds<PREC, NT, TH, staged>::total];
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  float2* lut = reinterpret_cast<float2*>(dyn);
  unsigned char* tab = dyn + 16 * (size_t)t_max;
  int lut_t = -1;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    const JobDesc& job = jobs[w.x];
    fused_tile<PREC, NT, TH, INTEGER>(job, w.y, w.z, smem, tab, lut, job.T != lut_t);
    lut_t = job.T;
  }
}

template <int PREC, int NT, int TH, bool INTEGER>
hipError_t launch_t(const JobDesc& job, hipStream_t stream) {
  using G = Geo<PREC, NT>;
  static_assert(G::THREADS == kThreadsFor<PREC>, "launch bounds");
  dim3 grid((job.width + G::COLS - 1) / G::COLS, (job.height + TH - 1) / TH);
  const size_t dyn = dynamic_lds(job.T, job.F);
  constexpr bool staged = INTEGER && Lds<PREC, NT, TH, true>::fits;
  if (Lds<PREC, NT, TH, staged>::total + dyn > kLdsLimit) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL((fused_kernel<PREC, NT, TH, INTEGER>), grid, dim3(G::THREADS), dyn, stream, job);
  return hipGetLastError();
}

// true when the staged (integer) variant with TH rows fits LDS for this T
template <int PREC, int NT, int TH>
bool staged_fits(int T, int F) {
  return Lds<PREC, NT, TH, true>::fits && Lds<PREC, NT, TH, true>::total + dynamic_lds(T, F) <= kLdsLimit;
}

}  // namespace fused_detail

}  // namespace bf
