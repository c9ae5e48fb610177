// Box spatial kernel by running sums (Sec. 1: the box window; Algorithm 1's
// smoothing step for w = 1 on [-W, W]^2).
//
// For w = 1 the separable smoothing of a plane is two sliding sums, one add
// and one subtract per plane and pass, independent of W.  This kernel runs
// eq. (9) for integer images with float32 planes that way: per harmonic k,
// every gray level's four plane values (cos, sin, (f - c0) cos, (f - c0) sin
// of k w f) come from a float32 table, the row sums slide along each row in
// float64 and are stored as float32, the column sums slide down each column
// in float64, and the demodulation accumulates P and Q in float64.  Nothing
// is rounded below float32 and no partial sum runs in float32, so the result
// stays as close to the FP64 eq. (9) as the float32 MFMA path while doing
// O(1) work per plane and pixel instead of O(W).
//
// Tile: 64 output columns x 64 output rows per workgroup of 512 threads,
// W <= 24.  LDS: the staged gray levels (16-bit) of the haloed tile, the row
// sums of the tile's 64 + 2W rows (float4 per column), and (dynamic) the
// per-harmonic table and the cos/sin(pi m / T) table.
#include "bf_fused_impl.h"

namespace bf {
namespace box_detail {

using namespace fused_detail;

constexpr int kThreads = 512;
constexpr int kCols = 64;   // output columns per tile
constexpr int kRows = 64;   // output rows per tile
constexpr int kMaxW = 24;
constexpr int kHR = kRows + 2 * kMaxW;      // row-sum rows
constexpr int kHS = kCols + 1;              // float4 per row-sum row (one of padding)
constexpr int kFC = kCols + 2 * kMaxW + 2;  // staged columns (u16), even
constexpr size_t kStatic = sizeof(float4) * kHR * kHS + 2 * (size_t)kHR * kFC + 4 * (2 * BF_MAX_W + 1) + 12;

// dynamic LDS: the per-harmonic table [(F + 1) x 16 B], then cos/sin(pi m / T) [2T x 8 B]
inline size_t dynamic_bytes(int T, int F) { return 16 * (size_t)(F + 1) + 8 * 2 * (size_t)T; }

__device__ __forceinline__ double4 d4(float4 v) { return make_double4(v.x, v.y, v.z, v.w); }

// One 64 x 64 output tile at (X0, Y0), all harmonics.  Every thread calls it.
__device__ __forceinline__ void box_tile(const JobDesc& job, int X0, int Y0, unsigned char* smem, unsigned char* dyn,
                                         bool build_lut) {
  auto H = reinterpret_cast<float4(*)[kHS]>(smem);
  auto ft = reinterpret_cast<uint16_t(*)[kFC]>(smem + sizeof(float4) * kHR * kHS);
  float* w1s = reinterpret_cast<float*>(smem + sizeof(float4) * kHR * kHS + 2 * (size_t)kHR * kFC);
  float4* tab = reinterpret_cast<float4*>(dyn);
  float2* lut = reinterpret_cast<float2*>(dyn + 16 * (size_t)(job.F + 1));

  const int tid = threadIdx.x;
  const int W = job.W, T = job.T, K = job.K, F = job.F;
  const int H_img = job.height, W_img = job.width;
  const int R = kRows + 2 * W;           // rows of row sums this tile needs
  const float c0 = job.c0;

  for (int m = tid; m < (build_lut ? 2 * T : 0); m += kThreads) {
    double s, c;
    sincospi((double)m / (double)T, &s, &c);
    lut[m] = make_float2((float)c, (float)s);
  }
  for (int t = tid; t <= 2 * W; t += kThreads) w1s[t] = job.w1[t];
  // stage the haloed tile: rows Y0 - W .., columns X0 - W .., folded borders
  stage_tile<kThreads>(job.src, job.src_pitch, R, kCols + 2 * W, Y0 - W, X0 - W, H_img, W_img, [&](int r, int c, float v) {
    v = fminf(fmaxf(v, 0.f), (float)F);  // NaN -> 0; the flag promises integers in [0, F]
    ft[r][c] = (uint16_t)(int)v;
  });

  // row-sum thread: row hr, 16-column quarter hs; column-sum thread: column
  // vx, 8-row eighth vq
  constexpr int kSegC = kCols / 4, kSegR = kRows / 8;
  const int hr = tid >> 2, hs = tid & 3;
  const int vx = tid & 63, vq = tid >> 6;
  double P[kSegR], Q[kSegR];
#pragma unroll
  for (int i = 0; i < kSegR; ++i) P[i] = Q[i] = 0.0;
  const PhaseTab pt{lut, 2.f * (float)T, 1.f / (2.f * (float)T), 1.f / (float)T, 2 * T};

  for (int k = 0; k <= K; ++k) {
    __syncthreads();  // the lut and tile are staged; every thread is done with harmonic k - 1
    for (int f = tid; f <= F; f += kThreads) {
      const float m = reduce_2t((float)k * (float)f, pt);
      const float2 cs = lut[min(max((int)m, 0), 2 * T - 1)];
      const float v = (float)f - c0;
      tab[f] = make_float4(cs.x, cs.y, v * cs.x, v * cs.y);
    }
    __syncthreads();
    // ---- row sums: H[r][x] = sum over tile columns x .. x + 2W of row r.
    // Loads run in chunks of 8 ahead of the (serial) running sum.
    if (hr < R) {
      const int x0 = kSegC * hs;
      double4 a = make_double4(0.0, 0.0, 0.0, 0.0), b = a;
      for (int c = x0; c <= x0 + 2 * W; c += 8) {
        float4 e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = tab[ft[hr][min(c + u, x0 + 2 * W)]];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (c + u > x0 + 2 * W) break;
          double4& t = (u & 1) ? b : a;
          t.x += e[u].x; t.y += e[u].y; t.z += e[u].z; t.w += e[u].w;
        }
      }
      a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
      H[hr][x0] = make_float4((float)a.x, (float)a.y, (float)a.z, (float)a.w);
      for (int x = x0 + 1; x < x0 + kSegC; x += 8) {
        float4 ein[8], eout[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int xu = min(x + u, x0 + kSegC - 1);
          ein[u] = tab[ft[hr][xu + 2 * W]];
          eout[u] = tab[ft[hr][xu - 1]];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (x + u >= x0 + kSegC) break;
          a.x += (double)ein[u].x - (double)eout[u].x;
          a.y += (double)ein[u].y - (double)eout[u].y;
          a.z += (double)ein[u].z - (double)eout[u].z;
          a.w += (double)ein[u].w - (double)eout[u].w;
          H[hr][x + u] = make_float4((float)a.x, (float)a.y, (float)a.z, (float)a.w);
        }
      }
    }
    __syncthreads();
    // ---- column sums down column vx, demodulation at kSegR output rows
    {
      const int y0 = kSegR * vq;
      double4 a = make_double4(0.0, 0.0, 0.0, 0.0), b = a;
      for (int r = y0; r <= y0 + 2 * W; r += 8) {
        float4 e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = H[min(r + u, y0 + 2 * W)][vx];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (r + u > y0 + 2 * W) break;
          double4& t = (u & 1) ? b : a;
          t.x += e[u].x; t.y += e[u].y; t.z += e[u].z; t.w += e[u].w;
        }
      }
      a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w;
      const double dk = job.d[k];
#pragma unroll
      for (int i0 = 0; i0 < kSegR; i0 += 8) {
        float2 cs[8];
        float4 ein[8], eout[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const float4 t = tab[ft[y0 + i0 + u + W][vx + W]];
          cs[u] = make_float2(t.x, t.y);
          const int iu = min(i0 + u, kSegR - 2);
          ein[u] = H[y0 + iu + 2 * W + 1][vx];
          eout[u] = H[y0 + iu][vx];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int i = i0 + u;
          const double dc = dk * (double)cs[u].x, ds = dk * (double)cs[u].y;
          Q[i] = fma(dc, a.x, fma(ds, a.y, Q[i]));
          P[i] = fma(dc, a.z, fma(ds, a.w, P[i]));
          if (i < kSegR - 1) {
            a.x += (double)ein[u].x - (double)eout[u].x;
            a.y += (double)ein[u].y - (double)eout[u].y;
            a.z += (double)ein[u].z - (double)eout[u].z;
            a.w += (double)ein[u].w - (double)eout[u].w;
          }
        }
      }
    }
  }

  // divide and store; then re-evaluate the pixels whose denominator (per
  // unit-sum window) is small directly
  const double n2 = (double)(2 * W + 1) * (double)(2 * W + 1);
  const double tau = (double)Planes<BF_PLANES_FP32>::kRefineQ * n2;
  const int xo = X0 + vx;
  unsigned flags = 0;
#pragma unroll
  for (int i = 0; i < kSegR; ++i) {
    const int yo = Y0 + kSegR * vq + i;
    if (yo < H_img && xo < W_img) {
      job.dst[(size_t)yo * job.dst_pitch + xo] = (float)(P[i] / Q[i] + (double)c0);
      if (!(Q[i] >= tau)) flags |= 1u << i;
    }
  }
  refine_pooled(flags != 0, [&](auto&& emit) {
    for (unsigned m = flags; m; m &= m - 1) emit(kSegR * vq + __ffs(m) - 1, vx);
  }, job, X0, Y0, W, w1s, lut, reinterpret_cast<unsigned char*>(tab), 16 * (size_t)(F + 1), kThreads,
  [&](int r, int c) { return (int)ft[r][c]; });
  __syncthreads();  // the LDS of this tile may be reused by the caller
}

__global__ void __launch_bounds__(kThreads) box_kernel(const JobDesc job) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[kStatic];
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  box_tile(job, blockIdx.x * kCols, blockIdx.y * kRows, smem, dyn, true);
}

// persistent form over a cost-ordered item list (job, x0, y0, -); dynamic
// LDS sized for the largest T and F of the class
__global__ void __launch_bounds__(kThreads) box_batched_kernel(const JobDesc* __restrict__ jobs,
                                                               const int4* __restrict__ items, int n_items,
                                                               int f_max) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[kStatic];
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  int lut_t = -1, lut_f = -1;
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int4 w = items[it];
    const JobDesc& job = jobs[w.x];
    // the lut follows the table, whose length depends on F
    (void)f_max;
    box_tile(job, w.y, w.z, smem, dyn, job.T != lut_t || job.F != lut_f);
    lut_t = job.T;
    lut_f = job.F;
  }
}

}  // namespace box_detail

bool box_supported(const JobDesc& job) {
  return (job.flags & kJobBox) && (job.flags & BF_FLAG_INTEGER_INPUT) && job.W <= box_detail::kMaxW &&
         box_detail::kStatic + box_detail::dynamic_bytes(job.T, job.F) <= fused_detail::kLdsLimit;
}

hipError_t launch_box(const JobDesc& job, hipStream_t stream) {
  using namespace box_detail;
  dim3 grid((job.width + kCols - 1) / kCols, (job.height + kRows - 1) / kRows);
  hipLaunchKernelGGL(box_kernel, grid, dim3(kThreads), dynamic_bytes(job.T, job.F), stream, job);
  return hipGetLastError();
}

hipError_t launch_box_batched(const JobDesc* jobs, const int4* items, int n_items, int t_max, int f_max, int grid,
                              hipStream_t stream) {
  using namespace box_detail;
  if (n_items <= 0) return hipSuccess;
  const size_t dyn = dynamic_bytes(t_max, f_max);
  if (kStatic + dyn > fused_detail::kLdsLimit) return hipErrorInvalidConfiguration;
  int g = grid;
  if (g <= 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&box_batched_kernel),
                                                     kThreads, dyn) != hipSuccess || per_cu < 1)
      per_cu = 1;
    g = cus * per_cu;
  }
  g = g < n_items ? g : n_items;
  hipLaunchKernelGGL(box_batched_kernel, dim3(g), dim3(kThreads), dyn, stream, jobs, items, n_items, f_max);
  return hipGetLastError();
}

}  // namespace bf
