// Kernel templates of the fused matrix-core smoothing step (2D, C >= 8; see
// step_mfma.hip).  Included by the instantiation units step_mfma_i*.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

#include "internal.h"
#include "step_mfma.h"

namespace mcmg {

namespace {

typedef float sfloatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 sbf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short sf2bf(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}

// Output tile TX x TY per tile id; regions grow by one node per side per
// phase: R3 = tile, R2 = tile + 1 (u), R1 = tile + 2 (t), R0 = tile + 3 (e).
template <int TI> struct STile;
template <> struct STile<0> { static constexpr int TX = 16, TY = 4; };
template <> struct STile<1> { static constexpr int TX = 32, TY = 4; };
template <> struct STile<2> { static constexpr int TX = 32, TY = 8; };
template <> struct STile<3> { static constexpr int TX = 64, TY = 8; };

template <int TI, bool BF, int NCT>
struct SGeo {
  static constexpr int TX = STile<TI>::TX, TY = STile<TI>::TY;
  static constexpr int W0 = TX + 6, H0 = TY + 6, N0 = W0 * H0;
  static constexpr int W1 = TX + 4, H1 = TY + 4, N1 = W1 * H1;
  static constexpr int W2 = TX + 2, H2 = TY + 2, N2 = W2 * H2;
  static constexpr int N3 = TX * TY;
  static constexpr int KV = BF ? 8 : 1, ES = BF ? 2 : 4;
  static constexpr int NCOL = 16 * NCT;
};

// Direct global-to-LDS copy of 16 bytes per lane: lane l of the wave writes
// lds_wave + 16 l (lds_wave the same in every lane); inactive lanes write
// nothing.  Completion is counted by vmcnt of the issuing wave.
__device__ __forceinline__ void slds_copy16(gptr<const unsigned char> g, void* lds_wave) {
  __builtin_amdgcn_global_load_lds((gptr<void>)g, (__attribute__((address_space(3))) void*)lds_wave, 16, 0, 0);
}

// One phase: for the region's row tiles (16 consecutive region nodes each,
// split over the 4 waves in groups of GR), acc[a] = sum over K of
// A(src region, tap offsets) x B(weights of tensor a); then `epi` stores
// the results.  The global operands of the epilogue are fetched by `pre`,
// before the group's K loop when EARLY, so their latency overlaps it.  Weights stream
// through LDS in chunks of up to `kc` K-steps, laid out [a][4 ks rows][BROW]
// (chunk vector idx at byte 16 idx) and copied straight from global memory.
template <bool BF, int NCT, int NACC, int GR, bool EARLY, class Pre, class Epi>
__device__ __forceinline__ void sphase(const SArgs& A, const unsigned char* src, int srcW, int dstW,
                                       int ndst, gptr<const unsigned char> w0, gptr<const unsigned char> w1,
                                       unsigned char* wbuf, int kc, Pre pre, Epi epi) {
  constexpr int KV = BF ? 8 : 1, ES = BF ? 2 : 4;
  constexpr int BROW = NCT * 16 * KV;           // elements of one pair row of the weights
  constexpr int V16 = BROW * ES / 16;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int stride = A.cinp + (BF ? 8 : 1);
  const int cpv = A.cinp / KV;
  const int nsteps = A.nsteps, npairs = A.npairs, ncols = A.ncols;
  const int ntile = (ndst + 15) / 16;
  const int per_wave = (ntile + 3) / 4;
  const int ngroups = (per_wave + GR - 1) / GR;
  const bool resident = kc >= nsteps;            // all weights of the phase fit at once
  for (int g = 0; g < ngroups; ++g) {
    sfloatx4 acc[NACC][GR][NCT];
#pragma unroll
    for (int a = 0; a < NACC; ++a)
#pragma unroll
      for (int i = 0; i < GR; ++i)
#pragma unroll
        for (int t = 0; t < NCT; ++t) acc[a][i][t] = sfloatx4{0.f, 0.f, 0.f, 0.f};
    // source node of each of this lane's row tiles (A row li)
    int snode[GR];
    bool live[GR];
#pragma unroll
    for (int i = 0; i < GR; ++i) {
      const int tile = wave + 4 * (g * GR + i);
      live[i] = tile < ntile;
      int n = tile * 16 + li;
      if (n >= ndst) n = ndst - 1;
      if (n < 0) n = 0;
      const int hy = n / dstW, hx = n - hy * dstW;
      snode[i] = hy * srcW + hx;                 // tap (0, 0) of the halo-1 source
    }
    int sbase[GR];                               // LDS element offset of tap (0, 0)
#pragma unroll
    for (int i = 0; i < GR; ++i) sbase[i] = snode[i] * stride;
    PairWalk pw;
    pw.init(lg, cpv, npairs);
    // epilogue operands: lane (li, lg) holds rows 4 lg + rr of each tile,
    // column li; fetched before the K loop when EARLY (latency hidden behind
    // it), else after it (fewer registers live across the loop)
    float2 ops[GR][NCT][4];
    auto fetch_ops = [&]() {
#pragma unroll
      for (int i = 0; i < GR; ++i)
#pragma unroll
        for (int t = 0; t < NCT; ++t)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const int n = (wave + 4 * (g * GR + i)) * 16 + 4 * lg + rr;
            ops[i][t][rr] = (live[i] && n < ndst) ? pre(n, t * 16 + li) : make_float2(0.f, 0.f);
          }
    };
    if constexpr (EARLY) fetch_ops();
    for (int s0 = 0; s0 < nsteps; s0 += kc) {
      const int ks = (nsteps - s0) < kc ? (nsteps - s0) : kc;
      if (!resident || (g == 0 && s0 == 0)) {
        __syncthreads();                         // previous chunk consumed
        const int total = NACC * 4 * ks * V16;
        for (int base = wave * 64; base < total; base += 256) {
          const int idx = base + lane;
          if (idx < total) {
            const int a = idx / (4 * ks * V16), rem = idx % (4 * ks * V16);
            const int row = rem / V16, vv = rem % V16;
            slds_copy16((a ? w1 : w0) +
                            ((size_t)(4 * s0 + row) * ncols * KV) * ES + (size_t)vv * 16,
                        wbuf + (size_t)__builtin_amdgcn_readfirstlane(base) * 16);
          }
        }
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's copies are in LDS
        __syncthreads();
      }
      // Row tiles past the region (live false) are computed on a clamped,
      // valid node and discarded, so no branch splits a step's LDS reads.
      typedef typename std::conditional<BF, sbf16x8, float>::type Frag;
      // steps are loaded in order, so the pair walk advances once per call
      auto load = [&](int ss, Frag (&bfr)[NACC][NCT], Frag (&af)[GR]) {
        const int s = s0 + ss;
        int tap, cb;
        pw.take(tap, cb);
        const int aoff = ((tap / 3) * srcW + (tap % 3)) * stride + cb * KV;
        const int wrow = resident ? s : ss;
#pragma unroll
        for (int a = 0; a < NACC; ++a)
#pragma unroll
          for (int t = 0; t < NCT; ++t) {
            const size_t o = ((size_t)a * 4 * ks + 4 * wrow + lg) * BROW + (t * 16 + li) * KV;
            if constexpr (BF) bfr[a][t] = *reinterpret_cast<const sbf16x8*>(reinterpret_cast<const unsigned short*>(wbuf) + o);
            else bfr[a][t] = reinterpret_cast<const float*>(wbuf)[o];
          }
#pragma unroll
        for (int i = 0; i < GR; ++i) {
          if constexpr (BF) af[i] = *reinterpret_cast<const sbf16x8*>(reinterpret_cast<const unsigned short*>(src) + sbase[i] + aoff);
          else af[i] = reinterpret_cast<const float*>(src)[sbase[i] + aoff];
        }
      };
      auto mma = [&](const Frag (&bfr)[NACC][NCT], const Frag (&af)[GR]) {
#pragma unroll
        for (int i = 0; i < GR; ++i)
#pragma unroll
          for (int t = 0; t < NCT; ++t)
#pragma unroll
            for (int a = 0; a < NACC; ++a) {
              if constexpr (BF) acc[a][i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[a][t], acc[a][i][t], 0, 0, 0);
              else acc[a][i][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bfr[a][t], acc[a][i][t], 0, 0, 0);
            }
      };
      Frag b0[NACC][NCT], a0[GR];
      for (int ss = 0; ss < ks; ++ss) {
        load(ss, b0, a0);
        mma(b0, a0);
      }
    }
    if constexpr (!EARLY) fetch_ops();
#pragma unroll
    for (int i = 0; i < GR; ++i) {
      if (!live[i]) continue;
      const int tile = wave + 4 * (g * GR + i);
#pragma unroll
      for (int t = 0; t < NCT; ++t)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int n = tile * 16 + 4 * lg + rr;
          if (n < ndst) epi(n, t * 16 + li, acc[0][i][t][rr], acc[NACC - 1][i][t][rr], ops[i][t][rr]);
        }
    }
  }
}

// The fused step e' = e + Wsm * (s (.) (KS * (r - W*e - a (.) (KA*e)))) on one
// output tile; FIRST (e = 0): e' = Wsm * (s (.) (KS * r)).
template <int TI, bool BF, int NCT, int VAR>
__device__ __forceinline__ void mstep_body(const SArgs& A, const int vblk) {
  using G = SGeo<TI, BF, NCT>;
  constexpr int ES = G::ES;
  extern __shared__ __align__(16) unsigned char smem[];
  const int C = A.C, cinp = A.cinp;
  const int stride = cinp + (BF ? 8 : 1);
  const int NY = A.n.n[0], NX = A.n.n[1];
  const int ntiles = A.tiles_x * A.tiles_y;
  const int per = (ntiles + 7) / 8;
  const int tl = (vblk % 8) * per + vblk / 8;   // XCD-contiguous bands
  if (tl >= ntiles) return;
  const int x0 = (tl % A.tiles_x) * G::TX, y0 = (tl / A.tiles_x) * G::TY;
  // LDS: region buffers (R0 and R2 share storage: e is dead once t exists),
  // then the weight chunk buffer
  auto rbytes = [&](int n) { return (((size_t)n * stride * ES + 15) / 16) * 16; };
  unsigned char* b02 = smem;
  unsigned char* b1 = smem + (rbytes(G::N0) > rbytes(G::N2) ? rbytes(G::N0) : rbytes(G::N2));
  unsigned char* wbuf = b1 + rbytes(G::N1);
  const gptr<const float> gr = to_global<const float>(A.r), ga = to_global<const float>(A.a);
  const gptr<const float> gs = to_global<const float>(A.s), ge = to_global<const float>(A.e);
  const gptr<float> geo = to_global<float>(A.eo);
  auto inside = [&](int y, int x) { return x >= 0 && x < NX && y >= 0 && y < NY; };
  auto put = [&](unsigned char* buf, int node, int c, float v) {
    if constexpr (BF) reinterpret_cast<unsigned short*>(buf)[(size_t)node * stride + c] = sf2bf(v);
    else reinterpret_cast<float*>(buf)[(size_t)node * stride + c] = v;
  };
  // stage a FP32 field [nodes][C] on a region of width W, height H, halo h;
  // loads are issued in batches of SB per thread before any LDS store
  auto stage = [&](unsigned char* buf, gptr<const float> f, int W, int H, int h) {
    constexpr int SB = 8;
    const int ng = cinp / 4;
    const int total = W * H * ng;
    const bool vec4 = (C % 4) == 0;
    for (int base = threadIdx.x; base < total; base += 256 * SB) {
      float4 v[SB];
#pragma unroll
      for (int k = 0; k < SB; ++k) {
        v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        const int idx = base + k * 256;
        if (idx >= total) continue;
        const int node = idx / ng, c = (idx % ng) * 4;
        const int hy = node / W, hx = node - hy * W;
        const int gy = y0 - h + hy, gx = x0 - h + hx;
        if (inside(gy, gx) && c < C) {
          const gptr<const float> p = f + ((size_t)gy * NX + gx) * C + c;
          if (vec4) v[k] = gld((gptr<const float4>)p, 0);
          else {
            v[k].x = p[0];
            if (c + 1 < C) v[k].y = p[1];
            if (c + 2 < C) v[k].z = p[2];
            if (c + 3 < C) v[k].w = p[3];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < SB; ++k) {
        const int idx = base + k * 256;
        if (idx >= total) continue;
        const int node = idx / ng, c = (idx % ng) * 4;
        if constexpr (BF) {
          // four bf16 values in one 8-byte store (node rows are 16-byte
          // aligned, c is a multiple of 4)
          const unsigned lo = (unsigned)sf2bf(v[k].x) | ((unsigned)sf2bf(v[k].y) << 16);
          const unsigned hi = (unsigned)sf2bf(v[k].z) | ((unsigned)sf2bf(v[k].w) << 16);
          *reinterpret_cast<uint2*>(reinterpret_cast<unsigned short*>(buf) + (size_t)node * stride + c) = make_uint2(lo, hi);
        } else {
          put(buf, node, c, v[k].x); put(buf, node, c + 1, v[k].y); put(buf, node, c + 2, v[k].z); put(buf, node, c + 3, v[k].w);
        }
      }
    }
  };
  // row tiles per group of a phase: the register budget (8 accumulator
  // tiles per wave; 12 for phase 1 at 32 channels, whose few blocks all fit
  // on the chip at once, so that its wave share of three tiles is one
  // group), but no more than a wave's share of the region's tiles
  constexpr int CAP1 = NCT == 2 ? 3 : ((8 / (2 * NCT)) > 0 ? 8 / (2 * NCT) : 1);
  constexpr int CAP2 = (8 / NCT) > 0 ? 8 / NCT : 1;
  constexpr int PW1 = ((G::N1 + 15) / 16 + 3) / 4, PW2 = ((G::N2 + 15) / 16 + 3) / 4;
  constexpr int PW3 = ((G::N3 + 15) / 16 + 3) / 4;
  constexpr int GR1 = CAP1 < PW1 ? CAP1 : PW1;
  constexpr int GR2 = CAP2 < PW2 ? CAP2 : PW2;
  constexpr int GR3 = CAP2 < PW3 ? CAP2 : PW3;
  // narrow channel counts have many small blocks, where occupancy counts
  // more than the epilogue latency of one block
  constexpr bool EARLY = NCT >= 2;

  // ---- phase 1: t on R1 (FIRST: t = r)
  if (VAR == L1_FIRST) {
    stage(b1, gr, G::W1, G::H1, 2);
  } else {
    stage(b02, ge, G::W0, G::H0, 3);
    // (the chunk loop's first barrier orders the staging before any read)
    sphase<BF, NCT, 2, GR1, EARLY>(A, b02, G::W0, G::W1, G::N1, to_global<const unsigned char>(A.wW), to_global<const unsigned char>(A.wKA), wbuf, A.kc1,
        [&](int n, int c) {
          const int hy = n / G::W1, hx = n - hy * G::W1;
          const int gy = y0 - 2 + hy, gx = x0 - 2 + hx;
          float2 v = make_float2(0.f, 0.f);
          if (c < C && inside(gy, gx)) {
            const size_t o = ((size_t)gy * NX + gx) * C + c;
            v = make_float2(gr[o], ga[o]);
          }
          return v;
        },
        [&](int n, int c, float aw, float aka, float2 ra) {
          if (c >= cinp) return;
          const int hy = n / G::W1, hx = n - hy * G::W1;
          const int gy = y0 - 2 + hy, gx = x0 - 2 + hx;
          float v = 0.f;
          if (c < C && inside(gy, gx)) v = ra.x - aw - ra.y * aka;
          put(b1, n, c, v);
        });
  }
  __syncthreads();
  // ---- phase 2: u = s (.) (KS * t) on R2 (into the R0 storage)
  sphase<BF, NCT, 1, GR2, EARLY>(A, b1, G::W1, G::W2, G::N2, to_global<const unsigned char>(A.wKS), nullptr, wbuf, A.kc2,
      [&](int n, int c) {
        const int hy = n / G::W2, hx = n - hy * G::W2;
        const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
        float2 v = make_float2(0.f, 0.f);
        if (c < C && inside(gy, gx)) v.x = gs[((size_t)gy * NX + gx) * C + c];
        return v;
      },
      [&](int n, int c, float acc, float, float2 sv) {
        if (c >= cinp) return;
        const int hy = n / G::W2, hx = n - hy * G::W2;
        const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
        float v = 0.f;
        if (c < C && inside(gy, gx)) v = sv.x * acc;
        put(b02, n, c, v);
      });
  __syncthreads();
  // ---- phase 3: e' = e + Wsm * u on the tile
  sphase<BF, NCT, 1, GR3, EARLY>(A, b02, G::W2, G::TX, G::N3, to_global<const unsigned char>(A.wSM), nullptr, wbuf, A.kc2,
      [&](int n, int c) {
        const int hy = n / G::TX, hx = n - hy * G::TX;
        const int gy = y0 + hy, gx = x0 + hx;
        float2 v = make_float2(0.f, 0.f);
        if (VAR != L1_FIRST && c < C && inside(gy, gx)) v.x = ge[((size_t)gy * NX + gx) * C + c];
        return v;
      },
      [&](int n, int c, float acc, float, float2 ev) {
        const int hy = n / G::TX, hx = n - hy * G::TX;
        const int gy = y0 + hy, gx = x0 + hx;
        if (c >= C || !inside(gy, gx)) return;
        const size_t o = ((size_t)gy * NX + gx) * C + c;
        geo[o] = (VAR == L1_FIRST) ? acc : ev.x + acc;
      });
}

template <int TI, bool BF, int NCT, int VAR>
__global__ __launch_bounds__(256) void mstep_kernel(SArgs A) {
  mstep_body<TI, BF, NCT, VAR>(A, blockIdx.x);
}

template <int TI, bool BF, int NCT, int VAR>
__global__ __launch_bounds__(256) void mstep_kernel_batched(const SArgs* __restrict__ tab,
                                                            const int* __restrict__ pre, int np,
                                                            const int* __restrict__ frozen,
                                                            const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const SArgs A = tab[batch_entry(row, np, p)];
  mstep_body<TI, BF, NCT, VAR>(A, blockIdx.x - pre[p]);
}

template <int TI, bool BF, int NCT, int VAR>
hipError_t srun(const StepLaunch& l, const BatchLaunch* b, hipStream_t s) {
  const size_t lds = mstep_lds_bytes(l.tile, l.bf16, l.ncols / 16, l.cinp, l.kc1, l.kc2);
  if (b) {
    hipLaunchKernelGGL((mstep_kernel_batched<TI, BF, NCT, VAR>), dim3(b->total), dim3(256), lds, s,
                       (const SArgs*)b->tab, b->pre, b->np, b->frozen, b->row);
  } else {
    int nblk;
    const SArgs A = step_args(l, &nblk);
    hipLaunchKernelGGL((mstep_kernel<TI, BF, NCT, VAR>), dim3(nblk), dim3(256), lds, s, A);
  }
  return hipGetLastError();
}

template <bool BF>
hipError_t sdispatch(const StepLaunch& l, const BatchLaunch* b, hipStream_t s) {
#define SCASE(TI, NCT)                                                                   \
  if (l.tile == TI && l.ncols == 16 * NCT)                                               \
    return l.var == L1_FIRST ? srun<TI, BF, NCT, L1_FIRST>(l, b, s) : srun<TI, BF, NCT, L1_STEP>(l, b, s);
  SCASE(0, 1) SCASE(0, 2) SCASE(0, 4)
  SCASE(1, 1) SCASE(1, 2) SCASE(1, 4)
  SCASE(2, 1) SCASE(2, 2) SCASE(2, 4)
  SCASE(3, 1) SCASE(3, 2) SCASE(3, 4)
#undef SCASE
  return hipErrorInvalidValue;
}

}  // namespace

}  // namespace mcmg

#define MSTEP_UNIT(NAME, BF)                                                              \
  namespace mcmg {                                                                         \
  hipError_t NAME(const StepLaunch& l, const BatchLaunch* b, hipStream_t s) {             \
    return sdispatch<BF>(l, b, s);                                                         \
  }                                                                                        \
  }
