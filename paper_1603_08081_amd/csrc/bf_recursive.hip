// Eq. (9) with the spatial convolutions of Algorithm 1 done by Deriche's
// recursive Gaussian, the constant-time smoothing Sec. 2 cites.  Three
// launches, the harmonics k = 0..K side by side in the grid (blockIdx.y):
//   1. rows:    one lane per (image row, k, plane), 64 rows staged through
//               LDS together, modulates f into its plane of
//               (f - c0) cos, (f - c0) sin, cos, sin of k w f (w = pi / T,
//               c0 the centre of the gray-level range) and runs the
//               causal and anti-causal fourth-order recursions over the row
//               (half-sample symmetric extension), writing the row-smoothed
//               planes of harmonic k;
//   2. columns: one lane per (image column, k, share) runs the same
//               recursions down two row-smoothed planes and demodulates with
//               d_k: harmonic k's share of the numerator,
//               cos S((f - c0) cos) + sin S((f - c0) sin), or of the
//               denominator, cos S(cos) + sin S(sin), times d_k (the causal
//               and anti-causal halves of S demodulated one after the
//               other); the workgroup sums the shares of its four harmonics
//               and writes one share per group;
//   3. one lane per pixel sums the groups' shares in float64, divides and
//      adds c0.
// The recursions' state is float64; so are the phases: computed per pixel,
// or for integer images looked up in a table of cos and sin of pi m / T
// (m = k f mod 2T), float32 in the row pass and float64 in the column pass'
// demodulation; the row-smoothed planes between the launches
// are float32, the shares float64 (the denominator of a wide spatial kernel
// can be a small difference of much larger shares, which float32 shares would
// leave with errors above 1e-3 gray levels).  Centring f on c0 halves the
// magnitude of the weighted planes and so their rounding.  Reads run ahead
// of the recursion steps that use them (the row pass's I/O wavefronts one
// block ahead, the column lanes one batch of positions ahead), so that memory
// latency overlaps arithmetic.  The recursion coefficients come from the four
// poles of Deriche's two damped cosine/sine pairs (his published fit of
// exp(-x^2/2)):
// the causal half of the kernel is a sum of four one-pole terms, whose common
// denominator and numerator give the recursion, and the anti-causal half
// (n >= 1, run backwards) has numerator N(z) - g(0) D(z).  Scaled to unit sum.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>

#include "bf_internal.h"

namespace bf {
namespace {

constexpr int kLineThreads = 64;     // one wavefront of lines per workgroup
// Above this the poles of the fourth-order recursion come so close to 1 that
// its float64 rounding reaches 1e-5 of the signal per pass.
constexpr double kMaxSigmaRec = 256.0;
// Images (rows x row pitch) below this many elements: the kernels' byte
// offsets of float64 shares then fit in 32 bits.
constexpr size_t kMaxRecElems = (size_t)1 << 28;

struct RecCoef {
  double nc[4];   // causal numerator, x(i) .. x(i - 3)
  double na[5];   // anti-causal numerator, x(i + 1) .. x(i + 4) in [1..4]
  double dd[5];   // denominator 1, d1..d4 (same for both directions)
  int margin;     // samples of symmetric extension before and after the line
};

struct RecArgs {
  const float* src;
  float* dst;
  int height, width, src_pitch, dst_pitch;
  int T;
  int K;
  int integer;     // BF_FLAG_INTEGER_INPUT: phases from tables of cos/sin(pi m / T)
  int F;           // integer images: gray levels 0..F
  float c0;        // centre of the gray-level range
  RecCoef c;
  float* rows;     // [K + 1][4][height][width], row-smoothed planes
  int groups;      // groups of kColGroup harmonics, ceil((K + 1) / kColGroup)
  double* P;       // [groups][height][width], numerator shares of the groups
  double* Q;       // [groups][height][width], denominator shares of the groups
  double d[BF_MAX_K + 1];   // d_0..d_K
};

// Deriche's fit of exp(-x^2 / 2), x >= 0: two damped pairs
// (a cos(w x) + a' sin(w x)) e^{-b x}
constexpr double kFitCos[2] = {1.680, -0.6803};
constexpr double kFitSin[2] = {3.735, -0.2598};
constexpr double kFitDecay[2] = {1.783, 1.723};
constexpr double kFitFreq[2] = {0.6318, 1.997};

RecCoef recursion_coefficients(double sigma) {
  using cd = std::complex<double>;
  cd poles[4], res[4];
  for (int p = 0; p < 2; ++p) {
    const cd z = std::polar(std::exp(-kFitDecay[p] / sigma), kFitFreq[p] / sigma);
    const cd alpha(kFitCos[p], -kFitSin[p]);
    poles[2 * p] = z;
    poles[2 * p + 1] = std::conj(z);
    res[2 * p] = 0.5 * alpha;
    res[2 * p + 1] = 0.5 * std::conj(alpha);
  }
  // D(u) = prod (1 - p u), u = z^-1, lowest power first
  cd D[5] = {1.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = 0; j < 4; ++j)
    for (int m = j + 1; m >= 1; --m) D[m] -= poles[j] * D[m - 1];
  // N(u) = sum_j r_j prod_{m != j} (1 - p_m u)
  cd N[4] = {0.0, 0.0, 0.0, 0.0};
  for (int j = 0; j < 4; ++j) {
    cd t[4] = {1.0, 0.0, 0.0, 0.0};
    int deg = 0;
    for (int m = 0; m < 4; ++m) {
      if (m == j) continue;
      ++deg;
      for (int q = deg; q >= 1; --q) t[q] -= poles[m] * t[q - 1];
    }
    for (int q = 0; q < 4; ++q) N[q] += res[j] * t[q];
  }
  RecCoef c{};
  double sum_n = 0.0, sum_a = 0.0, sum_d = 0.0;
  const double g0 = N[0].real();
  for (int q = 0; q < 5; ++q) c.dd[q] = D[q].real();
  for (int q = 0; q < 4; ++q) c.nc[q] = N[q].real();
  c.na[0] = 0.0;
  for (int q = 1; q < 4; ++q) c.na[q] = c.nc[q] - g0 * c.dd[q];
  c.na[4] = -g0 * c.dd[4];
  for (int q = 0; q < 4; ++q) sum_n += c.nc[q];
  for (int q = 1; q < 5; ++q) sum_a += c.na[q];
  for (int q = 0; q < 5; ++q) sum_d += c.dd[q];
  const double total = (sum_n + sum_a) / sum_d;
  for (int q = 0; q < 4; ++q) c.nc[q] /= total;
  for (int q = 1; q < 5; ++q) c.na[q] /= total;
  // the slowest decay is e^{-b n / sigma}: beyond this the kernel is < 1e-12 of
  // its peak (the sum of the tail < 1e-10 of the signal at sigma = 256, far
  // below the float32 rounding of the planes between the passes); rounded up
  // to whole 32-position blocks so that the row pass's blocks inside the
  // image start on 16-byte boundaries
  c.margin = (static_cast<int>(std::ceil(sigma * 12.0 * std::log(10.0) / kFitDecay[1])) + 8 + 31) / 32 * 32;
  return c;
}

// half-sample symmetric extension of a line of length L, any index (the
// integer remainder only for indices more than a line length outside it)
__device__ __forceinline__ int fold(int i, int L) {
  if ((unsigned)i < (unsigned)L) return i;
  if (i < 0 && i >= -L) return -i - 1;
  if (i >= L && i < 2 * L) return 2 * L - 1 - i;
  const int P = 2 * L;
  int j = i % P;
  if (j < 0) j += P;
  return j < L ? j : P - 1 - j;
}

// cos and sin of k pi f / T, the product reduced mod 2T first
__device__ __forceinline__ void phase(float f, int k, int T, double* c, double* s) {
  double a = static_cast<double>(k) * static_cast<double>(f);
  a = fmod(a, 2.0 * T);
  sincospi(a / T, s, c);
}

// The row pass goes through LDS in blocks of 64 rows x kChunk positions,
// double-buffered.  Four compute wavefronts run the four planes of the
// block's rows (wavefront p: plane p, lane = row; the planes are independent
// recursions), and four I/O wavefronts move the blocks between memory and LDS
// (each for 16 of the rows; a transfer instruction covers 8 rows x kChunk
// consecutive positions as 16-byte reads and writes where the block lies
// inside the row, 2 rows x kChunk single floats elsewhere).  While the compute
// wavefronts run block b, the I/O wavefronts store block b - 1's planes,
// stage block b + 1 from the registers its reads landed in and start the
// reads of block b + 2, so that one barrier per block is the only wait a
// compute wavefront has for memory (the I/O wavefronts' waits for their
// reads and stores hold up nothing else).
constexpr int kChunk = 32;
constexpr int kTileStride = kChunk + 1;   // odd stride: a lane per row hits distinct banks
constexpr int kRowBlock = 64;             // rows of a workgroup (lanes of a compute wavefront)
constexpr int kIoWaves = 4;
constexpr int kRowThreads = (4 + kIoWaves) * kLineThreads;
constexpr int kIoRowsPerInst = kLineThreads / kChunk;               // 2 rows per transfer instruction
constexpr int kIoInsts = kRowBlock / kIoWaves / kIoRowsPerInst;      // 8 per I/O lane, plane and block
constexpr int kTileFloats = kRowBlock * kTileStride;
static_assert(kLineThreads % kChunk == 0 && kRowBlock % (kIoWaves * kIoRowsPerInst) == 0,
              "I/O transfers cover whole row segments");

// m = k f mod 2T for an integer image: f clamped to the gray levels 0..F the
// integer flag promises (k f < 2^18 then, exact in float32); the quotient
// estimate in float32 is off by at most one, which the two corrections take
// back, so m is exact and always in [0, 2T)
__device__ __forceinline__ int phase_index(float f, int k, int T2, float inv_t2, float fmax) {
  const int kf = k * static_cast<int>(fminf(fmaxf(f, 0.0f), fmax));
  int m = kf - T2 * static_cast<int>(static_cast<float>(kf) * inv_t2);
  m += m < 0 ? T2 : 0;
  m -= m >= T2 ? T2 : 0;
  return m;
}

// a float at a wave-uniform base plus a 32-bit byte offset: the global
// access takes the base in scalar registers and one vector register for the
// offset (the host keeps images below 2^28 elements, so that every offset of
// the recursive path fits)
__device__ __forceinline__ float ld_at(const float* base, uint32_t byte_off) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ __forceinline__ void st_at(float* base, uint32_t byte_off, float v) {
  *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
__device__ __forceinline__ double ld_at(const double* base, uint32_t byte_off) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + byte_off);
}
__device__ __forceinline__ void st_at(double* base, uint32_t byte_off, double v) {
  *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// The row pass of one workgroup (64 rows, harmonic blockIdx.y).  INTEGER:
// phases from the float32 table of cos/sin(pi m / T).
template <bool INTEGER>
__global__ void __launch_bounds__(kRowThreads) rec_rows_kernel(const RecArgs a) {
  __shared__ float ft[2][kTileFloats];       // f of the block
  __shared__ float ot[2][4 * kTileFloats];   // the four planes of the block
  extern __shared__ float2 cs_tab[];         // 2T entries (cos, sin) when INTEGER
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kLineThreads);
  const int lane = tid % kLineThreads;
  const int y0 = blockIdx.x * kRowBlock;
  const int k = blockIdx.y;
  const int L = a.width, M = a.c.margin;
  const int nrows = min(kRowBlock, a.height - y0);
  const size_t plane = (size_t)a.height * a.width;
  float* outk = a.rows + 4 * plane * k;
  const int T2 = 2 * a.T;
  if (INTEGER) {
    for (int m = tid; m < T2; m += kRowThreads) {
      double c, s;
      sincospi(static_cast<double>(m) / a.T, &s, &c);
      cs_tab[m] = make_float2(static_cast<float>(c), static_cast<float>(s));
    }
  }
  // blocks: causal pass b = 0 .. nb - 1 at positions -M + kChunk b ..;
  // anti-causal pass from the top, block b at positions [lo, hi] with
  // hi = L - 1 + M - kChunk b, lo = max(hi - kChunk + 1, 0)
  const int nb = (L + M + kChunk - 1) / kChunk;
  auto causal_i0 = [&](int b) { return -M + kChunk * b; };
  auto anti_lo = [&](int b) { return max(L + M - kChunk * (b + 1), 0); };
  auto anti_n = [&](int b) { return L - 1 + M - kChunk * b - anti_lo(b) + 1; };

  if (wave >= 4) {
    // ---- I/O wavefront h: rows r0 + kIoRowsPerInst t (r0 = 16 h + lane / kChunk),
    // position q of the block, one float per lane and row (the scalar form)
    const int h = wave - 4;
    const int q = lane % kChunk, r0 = h * (kRowBlock / kIoWaves) + lane / kChunk;
    // byte offsets of row r0 + kIoRowsPerInst t in f and in a plane (rows past
    // the image are never accessed: row_ok masks them)
    const uint32_t s_row0 = 4u * static_cast<uint32_t>((y0 + r0) * a.src_pitch),
                   s_step = 4u * static_cast<uint32_t>(kIoRowsPerInst * a.src_pitch);
    const uint32_t o_row0 = 4u * static_cast<uint32_t>((y0 + r0) * L),
                   o_step = 4u * static_cast<uint32_t>(kIoRowsPerInst * L);
    auto srow = [&](int t) { return s_row0 + static_cast<uint32_t>(t) * s_step; };
    auto orow = [&](int t) { return o_row0 + static_cast<uint32_t>(t) * o_step; };
    auto row_ok = [&](int t) { return r0 + kIoRowsPerInst * t < nrows; };
    // float4 form of a block that lies inside the row and starts on a
    // 16-byte boundary: lane = (row rv0 + kRowsV t, quad c4 of 4 positions);
    // in both forms wavefront h moves the same 16 rows, so a block staged in
    // one form into the LDS buffer that another block, in the other form,
    // was just fetched from touches only this wavefront's elements
    const bool vec_ok = (L % 4) == 0 && (a.src_pitch % 4) == 0 &&
                        (reinterpret_cast<uintptr_t>(a.src) % 16) == 0;
    const int c4 = lane % (kChunk / 4), rv0 = h * (kRowBlock / kIoWaves) + lane / (kChunk / 4);
    constexpr int kRowsV = kLineThreads / (kChunk / 4);          // 8 rows per float4 instruction
    constexpr int kInstV = kRowBlock / kIoWaves / kRowsV;         // 2 per lane, plane and block
    static_assert(kInstV * 4 == kIoInsts, "both forms hold the same values per lane");
    auto srowv = [&](int t) { return 4u * static_cast<uint32_t>((y0 + rv0 + kRowsV * t) * a.src_pitch); };
    auto orowv = [&](int t) { return 4u * static_cast<uint32_t>((y0 + rv0 + kRowsV * t) * L); };
    auto rowv_ok = [&](int t) { return rv0 + kRowsV * t < nrows; };
    auto ld4 = [&](const float* base, uint32_t off) {
      return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(base) + off);
    };
    auto st4 = [&](float* base, uint32_t off, float4 v) {
      *reinterpret_cast<float4*>(reinterpret_cast<char*>(base) + off) = v;
    };
    auto fast_c = [&](int b) { return vec_ok && causal_i0(b) >= 0 && causal_i0(b) + kChunk <= L; };
    auto fast_a = [&](int b) { return vec_ok && anti_n(b) == kChunk && anti_lo(b) + kChunk <= L; };
    float fv[kIoInsts], ov[4][kIoInsts];
    // reads of causal block b (f at the block's position q)
    auto read_causal = [&](int b) {
      if (fast_c(b)) {
        const uint32_t col = 4u * static_cast<uint32_t>(causal_i0(b) + 4 * c4);
#pragma unroll
        for (int t = 0; t < kInstV; ++t) {
          const float4 v = rowv_ok(t) ? ld4(a.src, srowv(t) + col) : make_float4(0.f, 0.f, 0.f, 0.f);
          fv[4 * t] = v.x, fv[4 * t + 1] = v.y, fv[4 * t + 2] = v.z, fv[4 * t + 3] = v.w;
        }
        return;
      }
      const int i = causal_i0(b) + q;
      const bool ok = q < min(kChunk, L - causal_i0(b));
      const uint32_t col = 4u * static_cast<uint32_t>(fold(i, L));
#pragma unroll
      for (int t = 0; t < kIoInsts; ++t) fv[t] = (ok && row_ok(t)) ? ld_at(a.src, srow(t) + col) : 0.f;
    };
    // reads of anti-causal block b: f and the four causal halves
    auto read_anti = [&](int b) {
      if (fast_a(b)) {
        const uint32_t col = 4u * static_cast<uint32_t>(anti_lo(b) + 4 * c4);
#pragma unroll
        for (int t = 0; t < kInstV; ++t) {
          const bool ok = rowv_ok(t);
          const float4 v = ok ? ld4(a.src, srowv(t) + col) : make_float4(0.f, 0.f, 0.f, 0.f);
          fv[4 * t] = v.x, fv[4 * t + 1] = v.y, fv[4 * t + 2] = v.z, fv[4 * t + 3] = v.w;
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const float4 o = ok ? ld4(outk + p * plane, orowv(t) + col) : make_float4(0.f, 0.f, 0.f, 0.f);
            ov[p][4 * t] = o.x, ov[p][4 * t + 1] = o.y, ov[p][4 * t + 2] = o.z, ov[p][4 * t + 3] = o.w;
          }
        }
        return;
      }
      const int i = anti_lo(b) + q;
      const bool ok = q < anti_n(b);
      const uint32_t col = 4u * static_cast<uint32_t>(fold(i, L));
      const uint32_t pos = 4u * static_cast<uint32_t>(min(i, L - 1));
#pragma unroll
      for (int t = 0; t < kIoInsts; ++t) {
        fv[t] = (ok && row_ok(t)) ? ld_at(a.src, srow(t) + col) : 0.f;
#pragma unroll
        for (int p = 0; p < 4; ++p)
          ov[p][t] = (ok && row_ok(t) && i < L) ? ld_at(outk + p * plane, orow(t) + pos) : 0.f;
      }
    };
    auto stage = [&](int buf, bool planes, bool fast) {
      if (fast) {
#pragma unroll
        for (int t = 0; t < kInstV; ++t) {
          const int e0 = (rv0 + kRowsV * t) * kTileStride + 4 * c4;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            ft[buf][e0 + e] = fv[4 * t + e];
            if (planes) {
#pragma unroll
              for (int p = 0; p < 4; ++p) ot[buf][p * kTileFloats + e0 + e] = ov[p][4 * t + e];
            }
          }
        }
        return;
      }
#pragma unroll
      for (int t = 0; t < kIoInsts; ++t) {
        const int r = r0 + kIoRowsPerInst * t;
        ft[buf][r * kTileStride + q] = fv[t];
        if (planes) {
#pragma unroll
          for (int p = 0; p < 4; ++p) ot[buf][p * kTileFloats + r * kTileStride + q] = ov[p][t];
        }
      }
    };
    // the planes of a block from LDS to memory, positions i0 + q (< L, >= 0),
    // in two steps: fetch() reads them from LDS into registers, put() writes
    // them out, so that the staging of the next block (which waits for its
    // reads) can come between the two and not wait for these writes
    float sv[4][kIoInsts];
    auto fetch = [&](int buf, bool fast) {
      if (fast) {
#pragma unroll
        for (int t = 0; t < kInstV; ++t) {
          const int e0 = (rv0 + kRowsV * t) * kTileStride + 4 * c4;
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int p = 0; p < 4; ++p) sv[p][4 * t + e] = ot[buf][p * kTileFloats + e0 + e];
        }
        return;
      }
#pragma unroll
      for (int t = 0; t < kIoInsts; ++t) {
        const int r = r0 + kIoRowsPerInst * t;
#pragma unroll
        for (int p = 0; p < 4; ++p) sv[p][t] = ot[buf][p * kTileFloats + r * kTileStride + q];
      }
    };
    auto put = [&](int i0, int n, bool fast) {
      if (fast) {
        const uint32_t col = 4u * static_cast<uint32_t>(i0 + 4 * c4);
#pragma unroll
        for (int t = 0; t < kInstV; ++t) {
          if (!rowv_ok(t)) continue;
#pragma unroll
          for (int p = 0; p < 4; ++p)
            st4(outk + p * plane, orowv(t) + col,
                make_float4(sv[p][4 * t], sv[p][4 * t + 1], sv[p][4 * t + 2], sv[p][4 * t + 3]));
        }
        return;
      }
      const int i = i0 + q;
      if (q >= n || i < 0 || i >= L) return;
      const uint32_t pos = 4u * static_cast<uint32_t>(i);
#pragma unroll
      for (int t = 0; t < kIoInsts; ++t) {
        if (!row_ok(t)) continue;
#pragma unroll
        for (int p = 0; p < 4; ++p) st_at(outk + p * plane, orow(t) + pos, sv[p][t]);
      }
    };
    read_causal(0);
    stage(0, false, fast_c(0));
    if (nb > 1) read_causal(1);
    __syncthreads();
    for (int b = 0; b < nb; ++b) {
      if (b >= 1) fetch((b - 1) & 1, fast_c(b - 1));
      if (b + 1 < nb) {
        stage((b + 1) & 1, false, fast_c(b + 1));
        if (b + 2 < nb) read_causal(b + 2);
      }
      if (b >= 1) put(causal_i0(b - 1), min(kChunk, L - causal_i0(b - 1)), fast_c(b - 1));
      __syncthreads();
    }
    fetch((nb - 1) & 1, fast_c(nb - 1));
    put(causal_i0(nb - 1), min(kChunk, L - causal_i0(nb - 1)), fast_c(nb - 1));
    // the causal halves of every block are in memory before any is read back
    __syncthreads();
    read_anti(0);
    stage(0, true, fast_a(0));
    if (nb > 1) read_anti(1);
    __syncthreads();
    for (int b = 0; b < nb; ++b) {
      // (block b + 1 is staged into the buffer block b - 1 leaves: fetched first)
      if (b >= 1) fetch((b - 1) & 1, fast_a(b - 1));
      if (b + 1 < nb) {
        stage((b + 1) & 1, true, fast_a(b + 1));
        if (b + 2 < nb) read_anti(b + 2);
      }
      if (b >= 1) put(anti_lo(b - 1), anti_n(b - 1), fast_a(b - 1));
      __syncthreads();
    }
    fetch((nb - 1) & 1, fast_a(nb - 1));
    put(anti_lo(nb - 1), anti_n(nb - 1), fast_a(nb - 1));
    return;
  }

  // ---- compute wavefront: plane `wave` of row `lane`
  const int pl = wave;
  const double c0 = a.c0;
  const float inv_t2 = 1.0f / static_cast<float>(T2), fmax = static_cast<float>(a.F);
  const double pbase = pl < 2 ? 1.0 : 0.0;  // the plane carries (f - c0) for p < 2
  // plane pl of the modulated signal at gray level f:
  // (f - c0) cos, (f - c0) sin, cos, sin of k w f for pl = 0, 1, 2, 3
  auto modulated = [&](float f) -> double {
    double c, s;
    if constexpr (INTEGER) {
      const float2 cs = cs_tab[phase_index(f, k, T2, inv_t2, fmax)];
      c = cs.x;
      s = cs.y;
    } else {
      phase(f, k, a.T, &c, &s);
    }
    const double w = pbase != 0.0 ? (double)f - c0 : 1.0;
    return w * ((pl & 1) ? s : c);
  };
  const bool active = lane < nrows;
  // causal pass.  In a step the feedback terms come last, y(i-1)'s at the
  // very end, so that one step waits on the previous step's result for a
  // single multiply-add.
  double xh[4] = {};  // x(i), x(i-1), x(i-2), x(i-3)
  double yh[4] = {};  // y(i-1) .. y(i-4)
  auto causal_step = [&](double x) -> float {
    xh[3] = xh[2];
    xh[2] = xh[1];
    xh[1] = xh[0];
    xh[0] = x;
    const double ff = a.c.nc[0] * xh[0] + a.c.nc[1] * xh[1] + a.c.nc[2] * xh[2] + a.c.nc[3] * xh[3];
    const double v = ff - a.c.dd[4] * yh[3] - a.c.dd[3] * yh[2] - a.c.dd[2] * yh[1] - a.c.dd[1] * yh[0];
    yh[3] = yh[2];
    yh[2] = yh[1];
    yh[1] = yh[0];
    yh[0] = v;
    return static_cast<float>(v);
  };
  __syncthreads();
  for (int b = 0; b < nb; ++b) {
    const float* fr = ft[b & 1] + lane * kTileStride;
    float* orow_l = ot[b & 1] + pl * kTileFloats + lane * kTileStride;
    const int n = min(kChunk, L - causal_i0(b));
    if (active) {
      if (n == kChunk) {
#pragma unroll
        for (int j = 0; j < kChunk; ++j) orow_l[j] = causal_step(modulated(fr[j]));
      } else {
        for (int j = 0; j < n; ++j) orow_l[j] = causal_step(modulated(fr[j]));
      }
    }
    __syncthreads();
  }
  __syncthreads();
  // anti-causal pass: adds its half to the causal half in LDS
  double xa[4] = {};  // x(i+1) .. x(i+4)
  double ya[4] = {};  // y(i+1) .. y(i+4)
  auto anti_step = [&](double x) -> double {
    const double ff = a.c.na[1] * xa[0] + a.c.na[2] * xa[1] + a.c.na[3] * xa[2] + a.c.na[4] * xa[3];
    const double v = ff - a.c.dd[4] * ya[3] - a.c.dd[3] * ya[2] - a.c.dd[2] * ya[1] - a.c.dd[1] * ya[0];
    ya[3] = ya[2];
    ya[2] = ya[1];
    ya[1] = ya[0];
    ya[0] = v;
    xa[3] = xa[2];
    xa[2] = xa[1];
    xa[1] = xa[0];
    xa[0] = x;
    return v;
  };
  __syncthreads();
  for (int b = 0; b < nb; ++b) {
    const float* fr = ft[b & 1] + lane * kTileStride;
    float* orow_l = ot[b & 1] + pl * kTileFloats + lane * kTileStride;
    const int lo = anti_lo(b), n = anti_n(b);
    if (active) {
      if (n == kChunk && lo + kChunk <= L) {
#pragma unroll
        for (int j = kChunk - 1; j >= 0; --j)
          orow_l[j] = static_cast<float>(orow_l[j] + anti_step(modulated(fr[j])));
      } else {
        for (int j = n - 1; j >= 0; --j) {
          const double v = anti_step(modulated(fr[j]));
          if (lo + j < L) orow_l[j] = static_cast<float>(orow_l[j] + v);
        }
      }
    }
    __syncthreads();
  }
}

// The column pass demodulates the causal and the anti-causal halves of each
// smoothed plane separately (demodulation is linear), and sums the
// demodulated values of kColGroup harmonics inside the workgroup: the causal
// sweep writes the group's share of numerator or denominator at each pixel,
// and the anti-causal sweep adds the group's share of its own half, so that
// neither a causal half nor a per-harmonic share goes to memory.  Workgroup =
// kColGroup wavefronts, one harmonic each, lane = column; blockIdx.z picks
// the numerator share (planes 0 and 1) or the denominator share (planes 2
// and 3), so that each lane runs two recursions.  Each sweep reads
// kColAhead positions at a time, one batch ahead of the recursion steps;
// after a batch the wavefronts put their demodulated values in LDS and
// wavefront w sums positions w, w + kColGroup, ... of the batch over the
// group's harmonics in harmonic order.  For integer images the demodulation's cos and sin of
// pi m / T, m = k f mod 2T, come from a float64 table in LDS built by the
// workgroup.
constexpr int kColAhead = 8;
constexpr int kColGroup = 4;
constexpr int kColSums = kColAhead / kColGroup;  // positions of a batch each wavefront sums
static_assert(kColAhead % kColGroup == 0, "the wavefronts share a batch's sums evenly");
constexpr int kColThreads = kColGroup * kLineThreads;

__global__ void __launch_bounds__(kColThreads) rec_cols_kernel(const RecArgs a) {
  extern __shared__ double2 dcs_tab[];  // 2T entries (cos, sin) when a.integer
  __shared__ double red[2][kColGroup][kColAhead][kLineThreads];  // demodulated values of a batch
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kLineThreads);
  const int lane = tid % kLineThreads;
  const int x0 = blockIdx.x * kLineThreads + lane;
  const int grp = blockIdx.y;
  const int k = grp * kColGroup + wave;
  const bool kon = k <= a.K;        // wave-uniform: the last group may be short
  const bool xon = x0 < a.width;
  const bool on = kon && xon;
  const int half = blockIdx.z;  // 0: numerator share (planes 0, 1); 1: denominator share (planes 2, 3)
  if (a.integer) {
    for (int m = tid; m < 2 * a.T; m += kColThreads) {
      double c, s;
      sincospi(static_cast<double>(m) / a.T, &s, &c);
      dcs_tab[m] = make_double2(c, s);
    }
  }
  __syncthreads();
  const int T2 = 2 * a.T;
  const float inv_t2 = 1.0f / static_cast<float>(T2), fmax = static_cast<float>(a.F);
  // cos and sin of k pi f / T for this column's pixels
  const int kp = kon ? k : 0;  // (an idle wavefront's values are zero whatever its phases)
  auto demod_phase = [&](float f, double* c, double* s) {
    if (a.integer) {
      const double2 cs = dcs_tab[phase_index(f, kp, T2, inv_t2, fmax)];
      *c = cs.x;
      *s = cs.y;
    } else {
      phase(f, kp, a.T, c, s);
    }
  };
  const int L = a.height, M = a.c.margin, Wd = a.width;
  const size_t plane = (size_t)a.height * a.width;
  // wave-uniform bases; lane offsets in bytes
  const float* in0 = a.rows + (4 * (size_t)kp + 2 * half) * plane;
  const float* in1 = in0 + plane;
  double* share = (half ? a.Q : a.P) + plane * grp;  // the group's share
  const uint32_t xo = static_cast<uint32_t>(min(x0, Wd - 1));
  const double dk = kon ? a.d[k] : 0.0;
  // the sum over the group at position j of the batch in buffer buf
  auto group_sum = [&](int buf, int j) -> double {
    double acc = red[buf][0][j][lane];
#pragma unroll
    for (int h = 1; h < kColGroup; ++h) acc += red[buf][h][j][lane];
    return acc;
  };
  // the values of the next kColAhead positions are read while the current
  // ones run their recursion steps
  float nx[kColAhead][2], nf[kColAhead];
  double ns[kColSums] = {};  // the group's causal shares at this wavefront's positions of the next batch
  auto read_down = [&](int i0) {
#pragma unroll
    for (int j = 0; j < kColAhead; ++j) {
      const int i = i0 + j;
      const uint32_t r = 4u * (static_cast<uint32_t>(fold(i, L) * Wd) + xo);
      nx[j][0] = (on && i < L) ? ld_at(in0, r) : 0.f;
      nx[j][1] = (on && i < L) ? ld_at(in1, r) : 0.f;
      nf[j] = (on && i >= 0 && i < L) ? ld_at(a.src, 4u * (static_cast<uint32_t>(i * a.src_pitch) + xo)) : 0.f;
    }
  };
  double xh[2][4] = {};
  double yh[2][4] = {};
  read_down(-M);
  int it = 0;
  for (int i0 = -M; i0 < L; i0 += kColAhead, ++it) {
    float xin[kColAhead][2], fs[kColAhead];
#pragma unroll
    for (int j = 0; j < kColAhead; ++j) {
      xin[j][0] = nx[j][0];
      xin[j][1] = nx[j][1];
      fs[j] = nf[j];
    }
    if (i0 + kColAhead < L) read_down(i0 + kColAhead);
    const int buf = it & 1;
#pragma unroll
    for (int j = 0; j < kColAhead; ++j) {
      const int i = i0 + j;
      double sh = 0.0;
      if (i < L) {
        double S[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          xh[p][3] = xh[p][2];
          xh[p][2] = xh[p][1];
          xh[p][1] = xh[p][0];
          xh[p][0] = xin[j][p];
          const double ff = a.c.nc[0] * xh[p][0] + a.c.nc[1] * xh[p][1] + a.c.nc[2] * xh[p][2] +
                            a.c.nc[3] * xh[p][3];
          const double v = ff - a.c.dd[4] * yh[p][3] - a.c.dd[3] * yh[p][2] - a.c.dd[2] * yh[p][1] -
                           a.c.dd[1] * yh[p][0];
          yh[p][3] = yh[p][2];
          yh[p][2] = yh[p][1];
          yh[p][1] = yh[p][0];
          yh[p][0] = v;
          S[p] = v;
        }
        if (i >= 0) {
          double c, s;
          demod_phase(fs[j], &c, &s);
          sh = dk * (c * S[0] + s * S[1]);
        }
      }
      red[buf][wave][j][lane] = sh;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kColSums; ++u) {
      const int j = wave + kColGroup * u, i = i0 + j;
      if (xon && i >= 0 && i < L) st_at(share, 8u * (static_cast<uint32_t>(i * Wd) + xo), group_sum(buf, j));
    }
  }
  // (the group shares the upward sweep reads were written on the way down by
  // wavefronts of this workgroup, before at least one barrier)
  auto read_up = [&](int i0) {
#pragma unroll
    for (int j = 0; j < kColAhead; ++j) {
      const int i = i0 - j;
      const uint32_t r = 4u * (static_cast<uint32_t>(fold(i, L) * Wd) + xo);
      nx[j][0] = (on && i >= 0) ? ld_at(in0, r) : 0.f;
      nx[j][1] = (on && i >= 0) ? ld_at(in1, r) : 0.f;
      const bool out = i >= 0 && i < L;
      nf[j] = (on && out) ? ld_at(a.src, 4u * (static_cast<uint32_t>(i * a.src_pitch) + xo)) : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kColSums; ++u) {
      const int i = i0 - wave - kColGroup * u;
      ns[u] = (xon && i >= 0 && i < L) ? ld_at(share, 8u * (static_cast<uint32_t>(i * Wd) + xo)) : 0.0;
    }
  };
  double xa[2][4] = {};
  double ya[2][4] = {};
  read_up(L - 1 + M);
  for (int i0 = L - 1 + M; i0 >= 0; i0 -= kColAhead, ++it) {
    float xin[kColAhead][2], fs[kColAhead];
#pragma unroll
    for (int j = 0; j < kColAhead; ++j) {
      xin[j][0] = nx[j][0];
      xin[j][1] = nx[j][1];
      fs[j] = nf[j];
    }
    double so[kColSums];
#pragma unroll
    for (int u = 0; u < kColSums; ++u) so[u] = ns[u];
    if (i0 - kColAhead >= 0) read_up(i0 - kColAhead);
    const int buf = it & 1;
#pragma unroll
    for (int j = 0; j < kColAhead; ++j) {
      const int i = i0 - j;
      double sh = 0.0;
      if (i >= 0) {
        double S[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const double ff = a.c.na[1] * xa[p][0] + a.c.na[2] * xa[p][1] + a.c.na[3] * xa[p][2] +
                            a.c.na[4] * xa[p][3];
          const double v = ff - a.c.dd[4] * ya[p][3] - a.c.dd[3] * ya[p][2] - a.c.dd[2] * ya[p][1] -
                           a.c.dd[1] * ya[p][0];
          ya[p][3] = ya[p][2];
          ya[p][2] = ya[p][1];
          ya[p][1] = ya[p][0];
          ya[p][0] = v;
          xa[p][3] = xa[p][2];
          xa[p][2] = xa[p][1];
          xa[p][1] = xa[p][0];
          xa[p][0] = xin[j][p];
          S[p] = v;
        }
        if (i < L) {
          double c, s;
          demod_phase(fs[j], &c, &s);
          sh = dk * (c * S[0] + s * S[1]);
        }
      }
      red[buf][wave][j][lane] = sh;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kColSums; ++u) {
      const int j = wave + kColGroup * u, i = i0 - j;
      if (xon && i >= 0 && i < L) st_at(share, 8u * (static_cast<uint32_t>(i * Wd) + xo), so[u] + group_sum(buf, j));
    }
  }
}

// one lane per pixel: the group shares summed in group order, the division, + c0
__global__ void __launch_bounds__(256) rec_sum_kernel(const RecArgs a) {
  const size_t n = (size_t)a.height * a.width;
  const size_t o = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= n) return;
  double p = 0.0, q = 0.0;
  for (int g = 0; g < a.groups; ++g) {
    p += a.P[n * g + o];
    q += a.Q[n * g + o];
  }
  const int y = static_cast<int>(o / a.width), x = static_cast<int>(o % a.width);
  a.dst[(size_t)y * a.dst_pitch + x] = static_cast<float>(p / q + (double)a.c0);
}

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

int rec_groups(int K) { return (K + kColGroup) / kColGroup; }

// layout: row-smoothed planes of every harmonic (float32), numerator shares
// and denominator shares of every group of kColGroup harmonics (float64)
size_t rec_ws_bytes(int height, int width, int K) {
  const size_t n = (size_t)height * width, h = (size_t)K + 1, g = (size_t)rec_groups(K);
  return align256(4 * h * n * sizeof(float)) + 2 * align256(g * n * sizeof(double));
}

}  // namespace
}  // namespace bf

using namespace bf;

namespace {
// checks of the recursive path on top of resolve_job's; BF_OK or a negative status
int resolve_recursive(const bf_job* job, Resolved* r) {
  if (!job) return fail(BF_E_INVALID, "job is NULL");
  if (job->spatial != BF_SPATIAL_GAUSSIAN)
    return fail(BF_E_INVALID, "the recursive path smooths with a Gaussian: spatial must be BF_SPATIAL_GAUSSIAN");
  if (!(job->sigma_s > 0.0) || !std::isfinite(job->sigma_s))
    return fail(BF_E_INVALID, "sigma_s must be finite and > 0");
  if (job->sigma_s > kMaxSigmaRec) return fail(BF_E_UNSUPPORTED, "sigma_s exceeds 256");
  // the kernels address f, the planes and the shares with 32-bit byte offsets
  if (job->height >= 1 && job->width >= 1 &&
      (size_t)job->height * (size_t)std::max(job->src_pitch, job->width) >= kMaxRecElems)
    return fail(BF_E_UNSUPPORTED, "the recursive path takes images of fewer than 2^28 elements (rows x pitch)");
  // validation and fit shared with bf_filter; the window does not apply here
  bf_job j = *job;
  j.W = 0;
  return resolve_job(&j, r);
}
}  // namespace

extern "C" size_t bf_recursive_workspace_bytes(const bf_job* job) {
  Resolved r;
  if (resolve_recursive(job, &r) < 0) return (size_t)-1;
  return rec_ws_bytes(job->height, job->width, r.desc.K);
}

extern "C" int bf_filter_recursive(const bf_job* job, void* workspace, size_t ws_bytes, void* hip_stream) {
  Resolved r;
  const int rc = resolve_recursive(job, &r);
  if (rc < 0) return rc;
  const int K = r.desc.K;
  if (!workspace) return fail(BF_E_WORKSPACE, "workspace is NULL");
  if (ws_bytes < rec_ws_bytes(job->height, job->width, K))
    return fail(BF_E_WORKSPACE, "workspace smaller than bf_recursive_workspace_bytes()");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(BF_E_WORKSPACE, "workspace must be 256-byte aligned");
  const size_t n = (size_t)job->height * job->width, h = (size_t)K + 1;
  unsigned char* w = static_cast<unsigned char*>(workspace);
  RecArgs a{};
  a.src = job->src;
  a.dst = job->dst;
  a.height = job->height;
  a.width = job->width;
  a.src_pitch = job->src_pitch;
  a.dst_pitch = job->dst_pitch;
  a.T = job->T;
  a.integer = (job->flags & BF_FLAG_INTEGER_INPUT) ? 1 : 0;
  a.c0 = r.desc.c0;
  a.F = r.desc.F;
  a.c = recursion_coefficients(job->sigma_s);
  a.K = K;
  a.groups = rec_groups(K);
  const size_t planes = align256(4 * h * n * sizeof(float)),
               shares = align256((size_t)a.groups * n * sizeof(double));
  a.rows = reinterpret_cast<float*>(w);
  a.P = reinterpret_cast<double*>(w + planes);
  a.Q = reinterpret_cast<double*>(w + planes + shares);
  for (int k = 0; k <= K; ++k) a.d[k] = r.desc.d[k];
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  const dim3 grows((job->height + kRowBlock - 1) / kRowBlock, K + 1);
  const dim3 gcols((job->width + kLineThreads - 1) / kLineThreads, a.groups, 2);
  const size_t tab_bytes = a.integer ? 2 * (size_t)job->T * sizeof(float2) : 0;
  if (a.integer)
    hipLaunchKernelGGL(rec_rows_kernel<true>, grows, dim3(kRowThreads), tab_bytes, stream, a);
  else
    hipLaunchKernelGGL(rec_rows_kernel<false>, grows, dim3(kRowThreads), 0, stream, a);
  hipLaunchKernelGGL(rec_cols_kernel, gcols, dim3(kColThreads), a.integer ? 2 * (size_t)job->T * sizeof(double2) : 0,
                     stream, a);
  hipLaunchKernelGGL(rec_sum_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, a);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(BF_E_DEVICE, std::string("recursive-filter launch failed: ") + hipGetErrorString(e));
  return r.status;
}
