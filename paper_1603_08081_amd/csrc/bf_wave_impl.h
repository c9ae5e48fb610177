#pragma once
// Barrier-free tile kernel for 16-bit planes and integer gray levels.
//
// Same arithmetic as the shared-plane kernel in bf_fused_impl.h (eq. (9)
// through Algorithm 1 in its real cos/sin form), organised so that every wave
// works on its own: a wave owns a 16-column strip and builds the row-pass
// MFMA operands of its strip directly in registers from per-harmonic tables
// indexed by gray level, instead of reading planes that all waves wrote to
// LDS.  The only workgroup-wide synchronisation left is one barrier per
// harmonic (the tables are double-buffered by harmonic parity), so waves
// drift freely and the matrix, vector and LDS work of different waves
// overlaps.
//
// Per harmonic k and gray level f the modulation table holds the four plane
// values cos, sin, (f - c0) cos and (f - c0) sin of k w f, each rounded once
// to the plane format (8 bytes); the demodulation table holds d_k cos and
// d_k sin in fp32.  A row-pass operand is one 8-byte gather per pixel and
// two byte permutes per pixel pair and plane pair.
#include "bf_fused_impl.h"

namespace bf {
namespace fused_detail {

// (low 16 bits of a) | (low 16 bits of b) << 16, and the same for the high
// halves: one byte permute each (v_perm_b32 takes its second source as
// bytes 0-3 and its first as bytes 4-7)
__device__ __forceinline__ uint32_t lo_halves(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_perm(b, a, 0x05040100u);
}
__device__ __forceinline__ uint32_t hi_halves(uint32_t a, uint32_t b) {
  return __builtin_amdgcn_perm(b, a, 0x07060302u);
}

constexpr int kWaveNW = 8;                       // waves per workgroup
constexpr int kWaveThreads = 64 * kWaveNW;
constexpr int kWaveCols = 16 * kWaveNW;          // output columns per tile

template <int PREC, int NT>
struct WaveGeo {
  static constexpr int KS = (NT + 1) / 2;
  static constexpr int LWU = 16 * (kWaveNW - 1) + 32 * KS;  // staged input columns
  static constexpr int FW = LWU + 8;                         // padded row (u16)
  static constexpr int MODB = 8;                             // modulation-table entry bytes
};

// LDS use of one tile of TH rows: the gray-level table offsets of the staged tile
template <int PREC, int NT, int TH>
struct WaveLds {
  using G = WaveGeo<PREC, NT>;
  static constexpr int FROWS = 16 * (TH / 16 + NT - 1);
  static constexpr size_t tile = (size_t)FROWS * G::FW * 2;
  static constexpr size_t total = tile + 4 * (2 * BF_MAX_W + 1) + 64;
};

// dynamic LDS: cos/sin(pi m / T) [2T x 8 B], then the modulation tables
// [2][(T+1) x 8 B] and the demodulation tables [2][(T+1) x 8 B]
inline size_t wave_dynamic_lds(int T, int F) { return 32 * (size_t)(F + 1) + 16 * (size_t)T; }

// Wide-offset layout of the same kernel: the staged tile holds, per pixel,
// the 32-bit LDS byte address of its entry in the first modulation table, and
// the four tables (modulation and demodulation, two harmonic parities) sit at
// fixed 2 KB strides after it, so that a gather needs no address arithmetic:
// the table's offset is the LDS instruction's immediate.  It needs gray levels
// 0..255 and twice the staged-tile LDS; results are bit-identical to the
// 16-bit-offset layout.
constexpr int kWideSpan = 8 * 256;  // one table: 256 gray levels x 8 B
template <int PREC, int NT, int TH>
struct WideLds {
  using G = WaveGeo<PREC, NT>;
  static constexpr int FW = G::LWU + 4;  // padded row (u32)
  static constexpr int FROWS = 16 * (TH / 16 + NT - 1);
  static constexpr size_t tile = (size_t)FROWS * FW * 4;
  static constexpr size_t total = tile + 4 * (2 * BF_MAX_W + 1) + 64;
  using ReadAhead = TileReadAhead<kWaveThreads, FROWS, G::LWU>;  // one staged tile read ahead
};
// dynamic LDS of the wide layout: cos/sin(pi m / T) [2T x 8 B], then the four
// tables at kWideSpan strides
inline size_t wide_dynamic_lds(int T) { return 4 * (size_t)kWideSpan + 16 * (size_t)T; }

// reads at a 32-bit LDS byte address
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint2 lds_at_u2(uint32_t a) {
  const u32x2_t v = *(const __attribute__((address_space(3))) u32x2_t*)(size_t)a;
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ uint32_t lds_at_u1(uint32_t a) {
  return *(const __attribute__((address_space(3))) uint32_t*)(size_t)a;
}
__device__ __forceinline__ float2 lds_at_f2(uint32_t a) {
  const f32x2_t v = *(const __attribute__((address_space(3))) f32x2_t*)(size_t)a;
  return make_float2(v.x, v.y);
}

// One output tile (kWaveCols x TH at X0, Y0) of one image, all harmonics.
// tab has room for 4 (F+1) 8-byte entries; lut holds cos/sin(pi m / T),
// rebuilt here when build_lut is set.  Every thread of the workgroup must
// call it (it contains barriers).
template <int PREC, int NT, int TH>
__device__ __forceinline__ void wave_tile(const JobDesc& job, int X0, int Y0, uint16_t* ftile_raw, float* w1s,
                                          unsigned char* tab, float2* lut, bool build_lut) {
  using G = WaveGeo<PREC, NT>;
  using PT = Planes<PREC>;
  using E = typename PT::E;
  using RE = typename PT::RE;
  constexpr int KS = G::KS, LWU = G::LWU, FW = G::FW, MODB = G::MODB;
  constexpr int NJ = TH / 16, NS = NJ + NT - 1, FROWS = 16 * NS;
  auto ftile = reinterpret_cast<uint16_t(*)[FW]>(ftile_raw);

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, n16 = lane & 15;
  const int x0 = X0 + 16 * wave;
  const int W = job.W, T = job.T, K = job.K;
  const int Wal = (W + 7) & ~7;
  const int H = job.height, Wd = job.width;
  const float* __restrict__ src = job.src;
  const int sp = job.src_pitch;
  const float c0 = job.c0;
  const int F = job.F;
  const size_t span = 8 * (size_t)(F + 1);

  for (int m = tid; m < (build_lut ? 2 * T : 0); m += kWaveThreads) {
    double s, c;
    sincospi((double)m / (double)T, &s, &c);
    lut[m] = make_float2((float)c, (float)s);
  }
  for (int t = tid; t <= 2 * W; t += kWaveThreads) w1s[t] = job.w1[t];
  // stage the haloed tile once: folded borders, f clamped to [0, F]
  stage_tile<kWaveThreads>(src, sp, FROWS, LWU, Y0 - W, X0 - Wal, H, Wd, [&](int r, int c, float v) {
    v = fminf(fmaxf(v, 0.f), (float)F);  // NaN -> 0; the flag promises integers in [0, F]
    ftile[r][c] = (uint16_t)((int)v * MODB);
  });
  __syncthreads();

  auto wq = [&](int dd) -> float { return (dd >= -W && dd <= W) ? PT::round(w1s[dd + W]) : 0.f; };
  auto wqc = [&](int dd) -> float { return (dd >= -W && dd <= W) ? PT::round_col(w1s[dd + W]) : 0.f; };
  typename PT::V8 brow[KS];
  typename PT::RV8 bcol[KS];
  for (int ks = 0; ks < KS; ++ks)
    for (int e = 0; e < 8; ++e) {
      brow[ks][e] = (E)wq(32 * ks + 8 * g + e - Wal - n16);
      bcol[ks][e] = (RE)wqc(16 * (2 * ks + (e >> 2)) + 4 * g + (e & 3) - W - n16);
    }
  // k = 0: Q gains d_0 (sum of row weights) (sum of column weights)
  double wsum_r = 0.0, wsum_c = 0.0;
  for (int t = -W; t <= W; ++t) {
    wsum_r += (double)wq(t);
    wsum_c += (double)wqc(t);
  }
  const float q0 = (float)(job.d[0] * wsum_r * wsum_c);
  float P[NJ][4], Q[NJ][4];
  for (int j = 0; j < NJ; ++j)
    for (int i = 0; i < 4; ++i) P[j][i] = Q[j][i] = 0.f;

  const PhaseTab pt{lut, 2.f * (float)T, 1.f / (2.f * (float)T), 1.f / (float)T, 2 * T};
  auto tmod_k = [&](int kk) { return tab + (size_t)(kk & 1) * span; };
  auto tdem_k = [&](int kk) { return tab + (size_t)(2 + (kk & 1)) * span; };
  auto build = [&](int kk) {
    unsigned char* tm = tmod_k(kk);
    unsigned char* td = tdem_k(kk);
    const float dkf = (float)job.d[kk];
    for (int f = tid; f <= F; f += kWaveThreads) {
      const float m = reduce_2t((float)kk * (float)f, pt);
      const float2 cs = lut[min(max((int)m, 0), 2 * T - 1)];
      const float v = (float)f - c0;
      const uint32_t w0 = PT::bits(cs.x) | (PT::bits(cs.y) << 16);
      const uint32_t w1 = PT::bits(v * cs.x) | (PT::bits(v * cs.y) << 16);
      *reinterpret_cast<uint2*>(tm + MODB * f) = make_uint2(w0, w1);
      *reinterpret_cast<float2*>(td + 8 * f) = make_float2(dkf * cs.x, dkf * cs.y);
    }
  };

  build(0);
  if (K >= 1) build(1);
  for (int k = 0; k <= K; ++k) {
    __syncthreads();  // tables of harmonic k complete; every wave done with harmonic k - 1
    if (k >= 1 && k + 1 <= K) build(k + 1);
    const unsigned char* tm = tmod_k(k);
    const unsigned char* td = tdem_k(k);
    const float dk = (float)job.d[k];
    auto run = [&](auto nplc) {
      constexpr int NPL = decltype(nplc)::value;  // 1 for k = 0 (plane f - c0 only), else 4
      typename PT::RV4 ring[NT][NPL];
      // gray-level offsets of one step (read one step ahead) and, for the
      // four-plane harmonics, the gathered entries of two steps: the table
      // gathers of step s + 1 are issued before the permutes and MFMAs of
      // step s, so that their LDS latency hides behind them
      constexpr bool GPF = NPL == 4;
      uint4 fq_pf[KS];
      uint2 gd[GPF ? 2 : 1][GPF ? KS : 1][8];
      auto load_fq = [&](int step) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
          fq_pf[ks] = *reinterpret_cast<const uint4*>(&ftile[16 * step + n16][16 * wave + 32 * ks + 8 * g]);
      };
      auto gather = [&](int buf) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const uint4 fq = fq_pf[ks];
          const uint32_t fw[4] = {fq.x, fq.y, fq.z, fq.w};
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            gd[buf][ks][2 * h] = *reinterpret_cast<const uint2*>(tm + (fw[h] & 0xffffu));
            gd[buf][ks][2 * h + 1] = *reinterpret_cast<const uint2*>(tm + (fw[h] >> 16));
          }
        }
      };
      if constexpr (GPF) {
        load_fq(0);
        gather(0);
      }
      static_for<0, NS>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        if constexpr (GPF && s + 1 < NS) {
          load_fq(s + 1);
          gather((s + 1) & 1);
        }
        // ---- row pass of step s: operands gathered straight into registers
        f32x4 racc[NPL];
        for (int pi = 0; pi < NPL; ++pi) racc[pi] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int rr = 16 * s + n16, cc = 16 * wave + 32 * ks + 8 * g;
          typename PT::V8 a;
          if constexpr (NPL == 4) {
            uint32_t pc[4], ps[4], pfc[4], pfs[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {  // pixels 2h, 2h + 1
              const uint2 ta = gd[s & 1][ks][2 * h], tb = gd[s & 1][ks][2 * h + 1];
              pc[h] = lo_halves(ta.x, tb.x);
              ps[h] = hi_halves(ta.x, tb.x);
              pfc[h] = lo_halves(ta.y, tb.y);
              pfs[h] = hi_halves(ta.y, tb.y);
            }
            __builtin_memcpy(&a, pc, 16);
            racc[0] = PT::mma(a, brow[ks], racc[0]);
            __builtin_memcpy(&a, ps, 16);
            racc[1] = PT::mma(a, brow[ks], racc[1]);
            __builtin_memcpy(&a, pfc, 16);
            racc[2] = PT::mma(a, brow[ks], racc[2]);
            __builtin_memcpy(&a, pfs, 16);
            racc[3] = PT::mma(a, brow[ks], racc[3]);
          } else {
            // harmonic 0: the single plane f - c0
            const uint4 fq = *reinterpret_cast<const uint4*>(&ftile[rr][cc]);
            const uint32_t fw[4] = {fq.x, fq.y, fq.z, fq.w};
            uint32_t pv[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
              const float va = (float)((fw[h] & 0xffffu) / MODB) - c0;
              const float vb = (float)((fw[h] >> 16) / MODB) - c0;
              pv[h] = PT::bits(va) | (PT::bits(vb) << 16);
            }
            __builtin_memcpy(&a, pv, 16);
            racc[0] = PT::mma(a, brow[ks], racc[0]);
          }
        }
#pragma unroll
        for (int pi = 0; pi < NPL; ++pi) {
          typename PT::RV4 v;
          for (int i = 0; i < 4; ++i) v[i] = (RE)racc[pi][i];
          ring[s % NT][pi] = v;
        }
        // ---- column pass + demodulation of output tile j = s - NT + 1
        if constexpr (s >= NT - 1) {
          constexpr int j = s - NT + 1;
          float fb[NPL][4];
#pragma unroll
          for (int pi = 0; pi < NPL; ++pi) {
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            static_for<0, KS>([&](auto kc) {
              constexpr int ks = decltype(kc)::value;
              typename PT::RV4 lo = ring[(j + 2 * ks) % NT][pi];
              typename PT::RV4 hi;
              if constexpr (2 * ks + 1 < NT) hi = ring[(j + 2 * ks + 1) % NT][pi];
              else hi = typename PT::RV4{(RE)0.f, (RE)0.f, (RE)0.f, (RE)0.f};
              typename PT::RV8 a = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
              acc = PT::mma_col(a, bcol[ks], acc);
            });
            for (int i = 0; i < 4; ++i) fb[pi][i] = acc[i];
          }
          if constexpr (NPL == 4) {
            // table offsets of this lane's output pixels (row 16 j + n16,
            // columns 4 g .. 4 g + 3 of the strip), read from the tile
            const uint2 fo = *reinterpret_cast<const uint2*>(&ftile[W + 16 * j + n16][Wal + 16 * wave + 4 * g]);
            const uint32_t off[4] = {fo.x & 0xffffu, fo.x >> 16, fo.y & 0xffffu, fo.y >> 16};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float2 t = *reinterpret_cast<const float2*>(td + off[i]);
              P[j][i] = fmaf(t.x, fb[2][i], fmaf(t.y, fb[3][i], P[j][i]));
              Q[j][i] = fmaf(t.x, fb[0][i], fmaf(t.y, fb[1][i], Q[j][i]));
            }
          } else {
            for (int i = 0; i < 4; ++i) {
              P[j][i] = fmaf(dk, fb[0][i], P[j][i]);
              Q[j][i] += q0;
            }
          }
        }
      });
    };
    if (k == 0) run(std::integral_constant<int, 1>{});
    else run(std::integral_constant<int, 4>{});
  }

  float* __restrict__ dst = job.dst;
  for (int j = 0; j < NJ; ++j) {
    const int yy = Y0 + 16 * j + n16;
    if (yy >= H) continue;
    for (int i = 0; i < 4; ++i) {
      const int xx = x0 + 4 * g + i;
      if (xx < Wd) dst[(size_t)yy * job.dst_pitch + xx] = P[j][i] / Q[j][i] + c0;
    }
  }
  // re-evaluate ill-conditioned pixels directly (see refine_tile)
  const unsigned long long fl = refine_flags<NJ>(Q, job, Y0, x0, PT::kRefineQ);
  refine_tile<NJ>(fl, job, X0, Y0, Wal, w1s, lut, tab, 4 * span, kWaveThreads,
                  [&](int r, int c) { return (int)ftile[r][c] / MODB; });
  __syncthreads();  // the LDS of this tile may be reused by the caller
}

// wave_tile in the wide-offset layout (see WideLds): same arithmetic, same
// results.  tab points at the four tables (kWideSpan apart); the job's gray
// levels must lie in 0..255.  Harmonics run as odd/even pairs so that each
// body knows its table parity at compile time.
// ra: the reads of this tile when ra.valid (started by the previous tile), and
// on return those of the tile at (nX0, nY0) of *next when next is set.
template <int PREC, int NT, int TH>
__device__ __forceinline__ void wave_tile_wide(const JobDesc& job, int X0, int Y0, uint32_t* ftile_raw, float* w1s,
                                               unsigned char* tab, float2* lut, bool build_lut,
                                               typename WideLds<PREC, NT, TH>::ReadAhead& ra, const JobDesc* next,
                                               int nX0, int nY0) {
  using G = WaveGeo<PREC, NT>;
  using L = WideLds<PREC, NT, TH>;
  using PT = Planes<PREC>;
  using E = typename PT::E;
  using RE = typename PT::RE;
  constexpr int KS = G::KS, LWU = G::LWU, FW = L::FW, MODB = G::MODB, SPAN = kWideSpan;
  constexpr int NJ = TH / 16, NS = NJ + NT - 1, FROWS = 16 * NS;
  auto ftile = reinterpret_cast<uint32_t(*)[FW]>(ftile_raw);

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, g = lane >> 4, n16 = lane & 15;
  const int x0 = X0 + 16 * wave;
  const int W = job.W, T = job.T, K = job.K;
  const int Wal = (W + 7) & ~7;
  const int H = job.height, Wd = job.width;
  const float* __restrict__ src = job.src;
  const int sp = job.src_pitch;
  const float c0 = job.c0;
  const int F = job.F;
  const uint32_t tb = (uint32_t)(size_t)(__attribute__((address_space(3))) unsigned char*)tab;

  for (int m = tid; m < (build_lut ? 2 * T : 0); m += kWaveThreads) {
    double s, c;
    sincospi((double)m / (double)T, &s, &c);
    lut[m] = make_float2((float)c, (float)s);
  }
  for (int t = tid; t <= 2 * W; t += kWaveThreads) w1s[t] = job.w1[t];
  // stage the haloed tile once: folded borders, f clamped to [0, F], stored
  // as the address of the pixel's entry in the first modulation table
  auto put = [&](int r, int c, float v) {
    v = fminf(fmaxf(v, 0.f), (float)F);  // NaN -> 0; the flag promises integers in [0, F]
    ftile[r][c] = tb + (uint32_t)((int)v * MODB);
  };
  if (ra.valid) ra.commit(put);
  else stage_tile<kWaveThreads>(src, sp, FROWS, LWU, Y0 - W, X0 - Wal, H, Wd, put);
  __syncthreads();

  auto wq = [&](int dd) -> float { return (dd >= -W && dd <= W) ? PT::round(w1s[dd + W]) : 0.f; };
  auto wqc = [&](int dd) -> float { return (dd >= -W && dd <= W) ? PT::round_col(w1s[dd + W]) : 0.f; };
  typename PT::V8 brow[KS];
  typename PT::RV8 bcol[KS];
  for (int ks = 0; ks < KS; ++ks)
    for (int e = 0; e < 8; ++e) {
      brow[ks][e] = (E)wq(32 * ks + 8 * g + e - Wal - n16);
      bcol[ks][e] = (RE)wqc(16 * (2 * ks + (e >> 2)) + 4 * g + (e & 3) - W - n16);
    }
  // k = 0: Q gains d_0 (sum of row weights) (sum of column weights)
  double wsum_r = 0.0, wsum_c = 0.0;
  for (int t = -W; t <= W; ++t) {
    wsum_r += (double)wq(t);
    wsum_c += (double)wqc(t);
  }
  const float q0 = (float)(job.d[0] * wsum_r * wsum_c);
  float P[NJ][4], Q[NJ][4];
  for (int j = 0; j < NJ; ++j)
    for (int i = 0; i < 4; ++i) P[j][i] = Q[j][i] = 0.f;

  const PhaseTab pt{lut, 2.f * (float)T, 1.f / (2.f * (float)T), 1.f / (float)T, 2 * T};
  auto build = [&](int kk) {
    unsigned char* tm = tab + (size_t)(kk & 1) * SPAN;
    unsigned char* td = tab + (size_t)(2 + (kk & 1)) * SPAN;
    const float dkf = (float)job.d[kk];
    for (int f = tid; f <= F; f += kWaveThreads) {
      const float m = reduce_2t((float)kk * (float)f, pt);
      const float2 cs = lut[min(max((int)m, 0), 2 * T - 1)];
      const float v = (float)f - c0;
      const uint32_t w0 = PT::bits(cs.x) | (PT::bits(cs.y) << 16);
      const uint32_t w1 = PT::bits(v * cs.x) | (PT::bits(v * cs.y) << 16);
      *reinterpret_cast<uint2*>(tm + MODB * f) = make_uint2(w0, w1);
      *reinterpret_cast<float2*>(td + 8 * f) = make_float2(dkf * cs.x, dkf * cs.y);
    }
  };

  // one harmonic; NPL = 1 for k = 0 (plane f - c0 only), else 4; PAR = k & 1
  auto run = [&](auto nplc, auto parc) {
    constexpr int NPL = decltype(nplc)::value;
    constexpr int PAR = decltype(parc)::value;
    constexpr uint32_t MOFF = PAR * SPAN, DOFF = (2 + PAR) * SPAN;
    typename PT::RV4 ring[NT][NPL];
    constexpr bool GPF = NPL == 4;  // table gathers run one step ahead
    // entry addresses of one step (read one step ahead) and the gathered
    // entries of two steps (the gathers of step s + 1 are issued during step s)
    uint4 fq_pf[KS][2];
    uint2 gd[GPF ? 2 : 1][GPF ? KS : 1][8];
    auto load_fq = [&](int step) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const uint4* p = reinterpret_cast<const uint4*>(&ftile[16 * step + n16][16 * wave + 32 * ks + 8 * g]);
        fq_pf[ks][0] = p[0];
        fq_pf[ks][1] = p[1];
      }
    };
    auto gather = [&](int buf) {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const uint4 a0 = fq_pf[ks][0], a1 = fq_pf[ks][1];
        const uint32_t fw[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) gd[buf][ks][e] = lds_at_u2(fw[e] + MOFF);
      }
    };
    load_fq(0);
    if constexpr (GPF) gather(0);
    static_for<0, NS>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      if constexpr (GPF) {
        if constexpr (s + 1 < NS) {
          load_fq(s + 1);
          gather((s + 1) & 1);
        }
      }
      // ---- row pass of step s
      f32x4 racc[NPL];
      for (int pi = 0; pi < NPL; ++pi) racc[pi] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        typename PT::V8 a;
        if constexpr (NPL == 4) {
          uint32_t pc[4], ps[4], pfc[4], pfs[4];
#pragma unroll
          for (int h = 0; h < 4; ++h) {  // pixels 2h, 2h + 1
            const uint2 ta = gd[s & 1][ks][2 * h], tq = gd[s & 1][ks][2 * h + 1];
            pc[h] = lo_halves(ta.x, tq.x);
            ps[h] = hi_halves(ta.x, tq.x);
            pfc[h] = lo_halves(ta.y, tq.y);
            pfs[h] = hi_halves(ta.y, tq.y);
          }
          __builtin_memcpy(&a, pc, 16);
          racc[0] = PT::mma(a, brow[ks], racc[0]);
          __builtin_memcpy(&a, ps, 16);
          racc[1] = PT::mma(a, brow[ks], racc[1]);
          __builtin_memcpy(&a, pfc, 16);
          racc[2] = PT::mma(a, brow[ks], racc[2]);
          __builtin_memcpy(&a, pfs, 16);
          racc[3] = PT::mma(a, brow[ks], racc[3]);
        } else {
          // harmonic 0: the (f - c0) cos half of the harmonic-0 entry (cos = 1)
          if (ks == 0) load_fq(s);
          const uint4 a0 = fq_pf[ks][0], a1 = fq_pf[ks][1];
          const uint32_t fw[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
          uint32_t pv[4];
#pragma unroll
          for (int h = 0; h < 4; ++h)
            pv[h] = lo_halves(lds_at_u1(fw[2 * h] + MOFF + 4), lds_at_u1(fw[2 * h + 1] + MOFF + 4));
          __builtin_memcpy(&a, pv, 16);
          racc[0] = PT::mma(a, brow[ks], racc[0]);
        }
      }
#pragma unroll
      for (int pi = 0; pi < NPL; ++pi) {
        typename PT::RV4 v;
        for (int i = 0; i < 4; ++i) v[i] = (RE)racc[pi][i];
        ring[s % NT][pi] = v;
      }
      // ---- column pass + demodulation of output tile j = s - NT + 1
      if constexpr (s >= NT - 1) {
        constexpr int j = s - NT + 1;
        float fb[NPL][4];
#pragma unroll
        for (int pi = 0; pi < NPL; ++pi) {
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
          static_for<0, KS>([&](auto kc) {
            constexpr int ks = decltype(kc)::value;
            typename PT::RV4 lo = ring[(j + 2 * ks) % NT][pi];
            typename PT::RV4 hi;
            if constexpr (2 * ks + 1 < NT) hi = ring[(j + 2 * ks + 1) % NT][pi];
            else hi = typename PT::RV4{(RE)0.f, (RE)0.f, (RE)0.f, (RE)0.f};
            typename PT::RV8 a = __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
            acc = PT::mma_col(a, bcol[ks], acc);
          });
          for (int i = 0; i < 4; ++i) fb[pi][i] = acc[i];
        }
        if constexpr (NPL == 4) {
          // entry addresses of this lane's output pixels (row 16 j + n16,
          // columns 4 g .. 4 g + 3 of the strip) straight from the tile
          const uint4 o = *reinterpret_cast<const uint4*>(&ftile[W + 16 * j + n16][Wal + 16 * wave + 4 * g]);
          const uint32_t off[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float2 t = lds_at_f2(off[i] + DOFF);
            P[j][i] = fmaf(t.x, fb[2][i], fmaf(t.y, fb[3][i], P[j][i]));
            Q[j][i] = fmaf(t.x, fb[0][i], fmaf(t.y, fb[1][i], Q[j][i]));
          }
        } else {
          const float d0 = (float)job.d[0];
          for (int i = 0; i < 4; ++i) {
            P[j][i] = fmaf(d0, fb[0][i], P[j][i]);
            Q[j][i] += q0;
          }
        }
      }
    });
    // An empty asm that reads and writes P and Q: it keeps this harmonic's
    // demodulation inside its own body (otherwise the compiler sinks it past
    // the next barrier and spills the column-pass results).
#pragma unroll
    for (int j = 0; j < NJ; ++j)
      asm volatile("" : "+v"(P[j][0]), "+v"(P[j][1]), "+v"(P[j][2]), "+v"(P[j][3]), "+v"(Q[j][0]), "+v"(Q[j][1]),
                   "+v"(Q[j][2]), "+v"(Q[j][3]));
  };

  // tables of harmonic k at parity k & 1; the barrier before harmonic k also
  // releases the tables of k - 1, which the build of k + 1 then overwrites
  build(0);
  if (K >= 1) build(1);
  __syncthreads();
  run(std::integral_constant<int, 1>{}, std::integral_constant<int, 0>{});
  int k = 1;
  for (; k + 1 <= K; k += 2) {
    __syncthreads();
    build(k + 1);
    run(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{});
    __syncthreads();
    if (k + 2 <= K) build(k + 2);
    run(std::integral_constant<int, 4>{}, std::integral_constant<int, 0>{});
  }
  if (k <= K) {
    __syncthreads();
    run(std::integral_constant<int, 4>{}, std::integral_constant<int, 1>{});
  }
  float* __restrict__ dst = job.dst;
  for (int j = 0; j < NJ; ++j) {
    const int yy = Y0 + 16 * j + n16;
    if (yy >= H) continue;
    for (int i = 0; i < 4; ++i) {
      const int xx = x0 + 4 * g + i;
      if (xx < Wd) dst[(size_t)yy * job.dst_pitch + xx] = P[j][i] / Q[j][i] + c0;
    }
  }
  // re-evaluate ill-conditioned pixels directly (see refine_tile)
  const unsigned long long fl = refine_flags<NJ>(Q, job, Y0, x0, PT::kRefineQ);
  refine_tile<NJ>(fl, job, X0, Y0, Wal, w1s, lut, tab, 4 * (size_t)kWideSpan, kWaveThreads,
                  [&](int r, int c) { return (int)((ftile[r][c] - tb) >> 3); });
  // start reading the next tile (its block lands in registers while the
  // workgroup finishes this tile and sets up the next)
  // (ra.v is written on every path, so that the registers of a read never
  // committed are not kept across the next tile)
  {
    const int nWal = next ? (next->W + 7) & ~7 : 0;
    ra.valid = next && WideLds<PREC, NT, TH>::ReadAhead::eligible(next->src, next->src_pitch, nX0 - nWal, next->width);
    if (ra.valid) ra.issue(next->src, next->src_pitch, nY0 - next->W, nX0 - nWal, next->height);
    else ra.clear();
  }

  __syncthreads();  // the LDS of this tile may be reused by the caller
}

// variants whose staged tile cannot fit LDS even with the T = 255 tables are
// compiled empty and never launched (the host checks wave_fits / wide_fits)
template <int PREC, int NT, int TH>
constexpr bool kWaveBuildable =
    PREC != BF_PLANES_FP32 && WaveLds<PREC, NT, TH>::total + 32 * 256 + 16 * 255 <= kLdsLimit;
template <int PREC, int NT, int TH>
constexpr bool kWideBuildable =
    PREC != BF_PLANES_FP32 && WideLds<PREC, NT, TH>::total + 4 * kWideSpan + 16 * 255 <= kLdsLimit;

// one tile in the layout WIDE selects; dyn = dynamic LDS (cos/sin table of T
// entries pairs first, tables after it)
template <int PREC, int NT, int TH, bool WIDE>
__device__ __forceinline__ void wave_tile_any(const JobDesc& job, int X0, int Y0, void* ftile, float* w1s,
                                              unsigned char* dyn, int t_lut, bool build_lut,
                                              typename WideLds<PREC, NT, TH>::ReadAhead& ra,
                                              const JobDesc* next = nullptr, int nX0 = 0, int nY0 = 0) {
  float2* lut = reinterpret_cast<float2*>(dyn);
  unsigned char* tab = dyn + 16 * (size_t)t_lut;
  if constexpr (WIDE)
    wave_tile_wide<PREC, NT, TH>(job, X0, Y0, static_cast<uint32_t*>(ftile), w1s, tab, lut, build_lut, ra, next, nX0,
                                 nY0);
  else
    wave_tile<PREC, NT, TH>(job, X0, Y0, static_cast<uint16_t*>(ftile), w1s, tab, lut, build_lut);
}

template <int PREC, int NT, int TH, bool WIDE>
constexpr bool kLayoutBuildable = WIDE ? kWideBuildable<PREC, NT, TH> : kWaveBuildable<PREC, NT, TH>;

template <int PREC, int NT, int TH, bool WIDE>
__global__ void __launch_bounds__(kWaveThreads) wave_kernel(const JobDesc job) {
  if constexpr (kLayoutBuildable<PREC, NT, TH, WIDE>) {
    using Off = std::conditional_t<WIDE, uint32_t, uint16_t>;
    constexpr size_t TILE_ELEMS = WIDE ? (size_t)WideLds<PREC, NT, TH>::FROWS * WideLds<PREC, NT, TH>::FW
                                       : (size_t)WaveLds<PREC, NT, TH>::FROWS * WaveGeo<PREC, NT>::FW;
    __shared__ __attribute__((aligned(16))) Off ftile[TILE_ELEMS];
    __shared__ float w1s[2 * BF_MAX_W + 1];
    extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
    typename WideLds<PREC, NT, TH>::ReadAhead ra;
    ra.valid = false;
    wave_tile_any<PREC, NT, TH, WIDE>(job, blockIdx.x * kWaveCols, blockIdx.y * TH, ftile, w1s, dyn, job.T, true, ra);
  }
}

// Persistent form: workgroup b processes items b, b + gridDim.x, ... of a
// cost-ordered list; item = (job index, tile x0, tile y0, -).  Dynamic LDS is
// sized for T_max: cos/sin table first, then the per-harmonic tables.
template <int PREC, int NT, int TH, bool WIDE>
__global__ void __launch_bounds__(kWaveThreads) wave_batched_kernel(const JobDesc* __restrict__ jobs,
                                                                    const int4* __restrict__ items,
                                                                    int n_items, int t_max) {
  if constexpr (kLayoutBuildable<PREC, NT, TH, WIDE>) {
    using Off = std::conditional_t<WIDE, uint32_t, uint16_t>;
    constexpr size_t TILE_ELEMS = WIDE ? (size_t)WideLds<PREC, NT, TH>::FROWS * WideLds<PREC, NT, TH>::FW
                                       : (size_t)WaveLds<PREC, NT, TH>::FROWS * WaveGeo<PREC, NT>::FW;
    __shared__ __attribute__((aligned(16))) Off ftile[TILE_ELEMS];
    __shared__ float w1s[2 * BF_MAX_W + 1];
    extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
    int lut_t = -1;
    typename WideLds<PREC, NT, TH>::ReadAhead ra;
    ra.valid = false;
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
      const int4 w = items[it];
      const JobDesc& job = jobs[w.x];
      const bool more = it + (int)gridDim.x < n_items;
      const int4 nw = more ? items[it + gridDim.x] : make_int4(0, 0, 0, 0);
      wave_tile_any<PREC, NT, TH, WIDE>(job, w.y, w.z, ftile, w1s, dyn, t_max, job.T != lut_t, ra,
                                        more ? &jobs[nw.x] : nullptr, nw.y, nw.z);
      lut_t = job.T;
    }
  }
}

template <int PREC, int NT, int TH>
bool wave_fits(int T, int F) {
  return kWaveBuildable<PREC, NT, TH> && WaveLds<PREC, NT, TH>::total + wave_dynamic_lds(T, F) <= kLdsLimit;
}

// the wide layout: gray levels 0..255 (F <= 255) and the larger tile in LDS
template <int PREC, int NT, int TH>
bool wide_fits(int T, int F) {
  return kWideBuildable<PREC, NT, TH> && F <= 255 && WideLds<PREC, NT, TH>::total + wide_dynamic_lds(T) <= kLdsLimit;
}

template <int PREC, int NT, int TH>
hipError_t launch_wave(const JobDesc& job, hipStream_t stream) {
  dim3 grid((job.width + kWaveCols - 1) / kWaveCols, (job.height + TH - 1) / TH);
  if (!(job.flags & BF_FLAG_OFFSETS16) && wide_fits<PREC, NT, TH>(job.T, job.F))
    hipLaunchKernelGGL((wave_kernel<PREC, NT, TH, true>), grid, dim3(kWaveThreads), wide_dynamic_lds(job.T), stream,
                       job);
  else
    hipLaunchKernelGGL((wave_kernel<PREC, NT, TH, false>), grid, dim3(kWaveThreads), wave_dynamic_lds(job.T, job.F),
                       stream, job);
  return hipGetLastError();
}

// 96-, 128- and 144-row tiles (more output rows per halo row; 144 divides
// 2160-row frames into whole tiles) are built for windows up to W = 48; they
// may spill a few dozen registers to scratch, which costs less than the
// latency their longer software pipeline hides
template <int NT>
constexpr bool kWaveTall = NT <= 7;

template <int PREC, int NT, int TH>
bool wave_ok(int T, int F) {
  if constexpr (TH > 64 && !kWaveTall<NT>) return false;
  else return wave_fits<PREC, NT, TH>(T, F) || wide_fits<PREC, NT, TH>(T, F);
}

// Calls fn(integral_constant<int, TH>) for a wave-kernel tile height.
template <int NT, class F>
hipError_t with_wave_rows(int th, F&& fn) {
  if constexpr (kWaveTall<NT>) {
    if (th == 144) return fn(std::integral_constant<int, 144>{});
    if (th == 128) return fn(std::integral_constant<int, 128>{});
    if (th == 96) return fn(std::integral_constant<int, 96>{});
  }
  if (th == 64) return fn(std::integral_constant<int, 64>{});
  if (th == 32) return fn(std::integral_constant<int, 32>{});
  return hipErrorInvalidValue;
}

// Geometry and kernel family of one job: 16-bit planes on integer gray levels
// take the wave kernel with the tallest tile (<= th_pref) that fits; fp32
// planes the shared-plane kernel with a staged tile; the rest the general path.
template <int PREC, int NT>
TileChoice choose_tile(const JobDesc& job, int th_pref) {
  const bool integer = (job.flags & BF_FLAG_INTEGER_INPUT) != 0;
  const bool o16 = (job.flags & BF_FLAG_OFFSETS16) != 0;
  if constexpr (PREC != BF_PLANES_FP32) {
    if (integer) {
      if (th_pref >= 144 && wave_ok<PREC, NT, 144>(job.T, job.F)) return TileChoice{kWaveCols, 144, 1, o16};
      if (th_pref >= 128 && wave_ok<PREC, NT, 128>(job.T, job.F)) return TileChoice{kWaveCols, 128, 1, o16};
      if (th_pref >= 96 && wave_ok<PREC, NT, 96>(job.T, job.F)) return TileChoice{kWaveCols, 96, 1, o16};
      if (th_pref >= 64 && wave_ok<PREC, NT, 64>(job.T, job.F)) return TileChoice{kWaveCols, 64, 1, o16};
      if (wave_ok<PREC, NT, 32>(job.T, job.F)) return TileChoice{kWaveCols, 32, 1, o16};
    }
  } else if (integer) {
    if (th_pref >= 128 && staged_fits<PREC, NT, 128>(job.T, job.F)) return TileChoice{Geo<PREC, NT>::COLS, 128, 2, false};
    if (th_pref >= 96 && staged_fits<PREC, NT, 96>(job.T, job.F)) return TileChoice{Geo<PREC, NT>::COLS, 96, 2, false};
    if (th_pref >= 64 && staged_fits<PREC, NT, 64>(job.T, job.F)) return TileChoice{Geo<PREC, NT>::COLS, 64, 2, false};
    if (staged_fits<PREC, NT, 32>(job.T, job.F)) return TileChoice{Geo<PREC, NT>::COLS, 32, 2, false};
  }
  return TileChoice{Geo<PREC, NT>::COLS, 32, 0, false};
}

// One persistent launch over `n_items` items of one (family, TH) class.
template <int PREC, int NT>
hipError_t launch_batched_class(const JobDesc* jobs, const int4* items, int n_items, int t_max, int f_max,
                                TileChoice tc, int grid, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  auto fit_grid = [&](const void* fn, int threads, size_t dyn) {
    if (grid > 0) return min(grid, n_items);
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, dyn) != hipSuccess || per_cu < 1)
      per_cu = 1;
    return min(n_items, cus * per_cu);
  };
  if (tc.family == 1) {
    if constexpr (PREC == BF_PLANES_FP32) {
      return hipErrorInvalidValue;
    } else {
      return with_wave_rows<NT>(tc.th, [&](auto th_c) -> hipError_t {
        constexpr int TH = decltype(th_c)::value;
        if (!wave_ok<PREC, NT, TH>(t_max, f_max)) return hipErrorInvalidConfiguration;
        auto go = [&](auto wide_c, size_t dyn) -> hipError_t {
          constexpr bool WIDE = decltype(wide_c)::value;
          const void* fn = reinterpret_cast<const void*>(&wave_batched_kernel<PREC, NT, TH, WIDE>);
          const int g = fit_grid(fn, kWaveThreads, dyn);
          hipLaunchKernelGGL((wave_batched_kernel<PREC, NT, TH, WIDE>), dim3(g), dim3(kWaveThreads), dyn, stream,
                             jobs, items, n_items, t_max);
          return hipGetLastError();
        };
        if (!tc.offsets16 && wide_fits<PREC, NT, TH>(t_max, f_max)) return go(std::true_type{}, wide_dynamic_lds(t_max));
        return go(std::false_type{}, wave_dynamic_lds(t_max, f_max));
      });
    }
  }
  const size_t dyn = dynamic_lds(t_max, f_max);
  auto go = [&](auto th_c, auto int_c) -> hipError_t {
    constexpr int TH = decltype(th_c)::value;
    constexpr bool INT = decltype(int_c)::value;
    constexpr bool staged = INT && Lds<PREC, NT, TH, true>::fits;
    if (Lds<PREC, NT, TH, staged>::total + dyn > kLdsLimit) return hipErrorInvalidConfiguration;
    const int g = fit_grid(reinterpret_cast<const void*>(&fused_batched_kernel<PREC, NT, TH, INT>),
                           Geo<PREC, NT>::THREADS, dyn);
    hipLaunchKernelGGL((fused_batched_kernel<PREC, NT, TH, INT>), dim3(g), dim3(Geo<PREC, NT>::THREADS), dyn,
                       stream, jobs, items, n_items, t_max);
    return hipGetLastError();
  };
  if (tc.family == 2) {
    if constexpr (PREC == BF_PLANES_FP32) {
      if (tc.th == 128) return go(std::integral_constant<int, 128>{}, std::true_type{});
      if (tc.th == 96) return go(std::integral_constant<int, 96>{}, std::true_type{});
    }
    return tc.th == 64 ? go(std::integral_constant<int, 64>{}, std::true_type{})
                       : go(std::integral_constant<int, 32>{}, std::true_type{});
  }
  return go(std::integral_constant<int, 32>{}, std::false_type{});
}

}  // namespace fused_detail

// Kernel choice for one image: 16-bit planes on integer gray levels take the
// barrier-free kernel; fp32 planes take the shared-plane kernel with staged
// tile and tables; non-integer images (or tiles that would not fit LDS) take
// the general path of the shared-plane kernel.
template <int PREC, int NT>
hipError_t launch_fused_nt(const JobDesc& job, int th, hipStream_t stream) {
  using namespace fused_detail;
  const bool integer = (job.flags & BF_FLAG_INTEGER_INPUT) != 0;
  if constexpr (PREC != BF_PLANES_FP32) {
    if (integer) {
      const TileChoice tc = choose_tile<PREC, NT>(job, th);
      if (tc.family == 1)
        return with_wave_rows<NT>(tc.th, [&](auto th_c) { return launch_wave<PREC, NT, decltype(th_c)::value>(job, stream); });
    }
  } else if (integer) {
    if (th >= 128 && staged_fits<PREC, NT, 128>(job.T, job.F)) return launch_t<PREC, NT, 128, true>(job, stream);
    if (th >= 96 && staged_fits<PREC, NT, 96>(job.T, job.F)) return launch_t<PREC, NT, 96, true>(job, stream);
    if (th > 32 && staged_fits<PREC, NT, 64>(job.T, job.F)) return launch_t<PREC, NT, 64, true>(job, stream);
    if (staged_fits<PREC, NT, 32>(job.T, job.F)) return launch_t<PREC, NT, 32, true>(job, stream);
  }
  // general path; its per-pixel phase needs more registers, so 32-row tiles
  return launch_t<PREC, NT, 32, false>(job, stream);
}

}  // namespace bf
