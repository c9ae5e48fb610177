// Local dynamic range of an image (the T of Sec. 3 computed from the data):
// the largest |f(p) - f(q)| over pixel pairs whose offset lies in the window
// [-W, W]^2.  With the half-sample symmetric border of the filter, a folded
// neighbour of p is itself a pixel at most as far from p as the unfolded
// offset, so the folded window adds no new pairs and the value equals
//   max_p ( M(p) - f(p) ),  M = maximum of f over the window clipped to the image,
// which needs only a separable maximum filter.  Each 1-D running maximum is
// van Herk / Gil-Werman's: the staged line is cut into blocks of w = 2W + 1
// samples from its first staged sample, and within each block a prefix
// maximum g and a suffix maximum h are formed; a window [a, b] of at most w
// samples then has maximum max(h[a], g[b]) when a and b lie in different
// blocks, g[b] when a starts their common block and h[a] otherwise (b then
// ends the staged line), so each output costs O(1) whatever W.  Three launches:
//   1. rows:    R(y, x) = max f(y, x') over |x' - x| <= W (clipped), one
//               workgroup per row segment, the segment staged in LDS;
//   2. columns: M(y, x) = max R(y', x) over |y' - y| <= W (clipped) from an
//               LDS tile, then max (M - f) per workgroup;
//   3. one workgroup reduces the per-workgroup maxima and writes ceil(max).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "bf_internal.h"

namespace bf {
namespace {

constexpr int kRowSeg = 256;          // outputs per row workgroup
constexpr int kColW = 32;             // columns per column workgroup
constexpr int kColH = 64;             // output rows per column workgroup
constexpr int kColThreads = 256;      // 32 columns x 8 row groups

// Suffix (h) and prefix maxima of v[0..n) within blocks of w samples
// starting at 0, one block per thread at a time; the prefix maxima overwrite
// v (g = v on return); element i of a line is at stride `st` (1 along a row,
// the tile width down a column).
__device__ __forceinline__ void block_scans(float* v, float* h, int n, int w, int st, int lane0, int nlanes) {
  const int nb = (n + w - 1) / w;
  for (int bk = lane0; bk < nb; bk += nlanes) {
    const int s0 = bk * w, s1 = min(s0 + w, n);
    float m = v[(s1 - 1) * st];
    h[(s1 - 1) * st] = m;
    for (int i = s1 - 2; i >= s0; --i) {
      m = fmaxf(m, v[i * st]);
      h[i * st] = m;
    }
    m = v[s0 * st];
    for (int i = s0 + 1; i < s1; ++i) {
      m = fmaxf(m, v[i * st]);
      v[i * st] = m;
    }
  }
}

// maximum over staged samples [a, b] (b - a < w) from the block maxima
__device__ __forceinline__ float window_max(const float* g, const float* h, int a, int b, int w, int st) {
  const int ba = a / w, bb = b / w;
  if (ba != bb) return fmaxf(h[a * st], g[b * st]);
  return (a == ba * w) ? g[b * st] : h[a * st];
}

__global__ void __launch_bounds__(kRowSeg) row_max_kernel(const float* __restrict__ src, int H, int Wd, int pitch,
                                                          int W, float* __restrict__ rmax) {
  __shared__ float seg[kRowSeg + 2 * BF_MAX_W];  // the segment, then its prefix maxima
  __shared__ float hs[kRowSeg + 2 * BF_MAX_W];
  const int y = blockIdx.y;
  const int x0 = blockIdx.x * kRowSeg;
  const int lo = max(x0 - W, 0), hi = min(x0 + kRowSeg + W, Wd);  // staged [lo, hi)
  const int w = 2 * W + 1;
  for (int x = lo + (int)threadIdx.x; x < hi; x += kRowSeg) seg[x - lo] = src[(size_t)y * pitch + x];
  __syncthreads();
  block_scans(seg, hs, hi - lo, w, 1, (int)threadIdx.x, kRowSeg);
  __syncthreads();
  const int x = x0 + (int)threadIdx.x;
  if (x >= Wd) return;
  const int a = max(x - W, 0), b = min(x + W, Wd - 1);
  rmax[(size_t)y * Wd + x] = window_max(seg, hs, a - lo, b - lo, w, 1);
}

__global__ void __launch_bounds__(kColThreads) col_max_kernel(const float* __restrict__ src, int H, int Wd,
                                                              int pitch, int W, const float* __restrict__ rmax,
                                                              float* __restrict__ block_max) {
  extern __shared__ float tile[];  // two arrays of [(kColH + 2W) rows][kColW]: R (then its prefix maxima), suffix maxima
  __shared__ float red[kColThreads];
  const int x0 = blockIdx.x * kColW, y0 = blockIdx.y * kColH;
  const int r_lo = max(y0 - W, 0), r_hi = min(y0 + kColH + W, H);
  const int nr = r_hi - r_lo, w = 2 * W + 1;
  float* ht = tile + (size_t)(kColH + 2 * W) * kColW;
  const int c = threadIdx.x & (kColW - 1), grp = threadIdx.x / kColW;
  const int x = x0 + c;
  for (int r = r_lo + grp; r < r_hi; r += kColThreads / kColW)
    tile[(r - r_lo) * kColW + c] = (x < Wd) ? rmax[(size_t)r * Wd + x] : 0.f;
  __syncthreads();
  // the row groups share a column's blocks
  block_scans(tile + c, ht + c, nr, w, kColW, grp, kColThreads / kColW);
  __syncthreads();
  float best = 0.f;
  if (x < Wd) {
    for (int y = y0 + grp; y < min(y0 + kColH, H); y += kColThreads / kColW) {
      const int a = max(y - W, 0), b = min(y + W, H - 1);
      const float m = window_max(tile + c, ht + c, a - r_lo, b - r_lo, w, kColW);
      best = fmaxf(best, m - src[(size_t)y * pitch + x]);
    }
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int s = kColThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) block_max[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) final_max_kernel(const float* __restrict__ block_max, int n, int* T_out) {
  __shared__ float red[256];
  float m = 0.f;
  for (int i = threadIdx.x; i < n; i += 256) m = fmaxf(m, block_max[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) T_out[0] = (int)ceilf(red[0]);
}

size_t n_col_blocks(int H, int Wd) {
  return (size_t)((Wd + kColW - 1) / kColW) * (size_t)((H + kColH - 1) / kColH);
}

size_t range_ws_bytes(int H, int Wd) {
  const size_t r = (sizeof(float) * (size_t)H * Wd + 255) / 256 * 256;
  return r + sizeof(float) * n_col_blocks(H, Wd);
}

}  // namespace
}  // namespace bf

using namespace bf;

extern "C" size_t bf_dynamic_range_workspace_bytes(int height, int width) {
  if (height < 1 || width < 1) return (size_t)-1;
  return range_ws_bytes(height, width);
}

extern "C" int bf_dynamic_range(const float* src, int height, int width, int src_pitch, int W, int* T_out,
                                void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!src || !T_out) return fail(BF_E_INVALID, "src and T_out must be device pointers");
  if (height < 1 || width < 1) return fail(BF_E_INVALID, "height and width must be >= 1");
  if (src_pitch < width) return fail(BF_E_INVALID, "pitch must be >= width");
  if (W < 0 || W > BF_MAX_W) return fail(BF_E_INVALID, "W must satisfy 0 <= W <= BF_MAX_W");
  if (!workspace) return fail(BF_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < range_ws_bytes(height, width))
    return fail(BF_E_WORKSPACE, "workspace smaller than bf_dynamic_range_workspace_bytes()");
  if (reinterpret_cast<uintptr_t>(workspace) % 16 != 0) return fail(BF_E_WORKSPACE, "workspace must be 16-byte aligned");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  float* rmax = static_cast<float*>(workspace);
  float* bmax = reinterpret_cast<float*>(static_cast<unsigned char*>(workspace) +
                                         (sizeof(float) * (size_t)height * width + 255) / 256 * 256);
  const dim3 g1((width + kRowSeg - 1) / kRowSeg, height);
  hipLaunchKernelGGL(row_max_kernel, g1, dim3(kRowSeg), 0, stream, src, height, width, src_pitch, W, rmax);
  const dim3 g2((width + kColW - 1) / kColW, (height + kColH - 1) / kColH);
  const size_t lds = 2 * sizeof(float) * (size_t)(kColH + 2 * W) * kColW;
  hipLaunchKernelGGL(col_max_kernel, g2, dim3(kColThreads), lds, stream, src, height, width, src_pitch, W, rmax,
                     bmax);
  const int nb = static_cast<int>(n_col_blocks(height, width));
  hipLaunchKernelGGL(final_max_kernel, dim3(1), dim3(256), 0, stream, bmax, nb, T_out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(BF_E_DEVICE, std::string("dynamic-range launch failed: ") + hipGetErrorString(e));
  return BF_OK;
}
