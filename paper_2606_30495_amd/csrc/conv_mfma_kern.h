// Kernel templates of the matrix-core convolutions (included by the
// per-(dim, precision, mode group) instantiation units conv_mfma_i*.hip; the
// algorithm is described in conv_mfma.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <type_traits>

#include "conv_mfma.h"
#include "internal.h"

namespace mcmg {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

// Direct global-to-LDS copy of 16 bytes per lane: lane l of the wave writes
// lds_wave + 16 l (lds_wave must be the same in every lane); inactive lanes
// write nothing.  Completion is counted by vmcnt of the issuing wave.
__device__ __forceinline__ void lds_copy16(gptr<const unsigned char> g, void* lds_wave) {
  __builtin_amdgcn_global_load_lds((gptr<void>)g, (__attribute__((address_space(3))) void*)lds_wave, 16, 0, 0);
}

__device__ __forceinline__ u16 f2bf(float f) {
  unsigned int u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (u16)(u >> 16);
}

// Output tile and staged input tile geometry per (D, MODE, MT, RPW): the
// block's 4 * RPW GEMM rows (node rows along y, z) are split over its 4
// waves, row rho = wave + 4 i (i < RPW); each row holds 16 * MT nodes in x.
template <int D, int MODE, int MT, int RPW>
struct Geo {
  static constexpr int TX = 16 * MT;
  static constexpr int ROWS = 4 * RPW;
  static constexpr int TY = (D == 2) ? ROWS : (RPW == 1 ? 2 : 4);
  static constexpr int TZ = (D == 2) ? 1 : ROWS / TY;
  // staged tile extent per axis
  static constexpr int ext(int t) { return MODE == CONV_S1 ? t + 2 : (MODE == CONV_S2 ? 2 * t + 1 : t + 1); }
  static constexpr int HX = ext(TX), HY = ext(TY), HZ = (D == 2) ? 1 : ext(TZ);
  static constexpr int NODES = HX * HY * HZ;
  static constexpr int TAPS = (MODE == CONV_T2) ? ((D == 2) ? 4 : 8) : ((D == 2) ? 9 : 27);
  static constexpr int W = (MODE == CONV_T2) ? 2 : 3;   // window per axis
};

template <bool BF> constexpr int KVOF() { return BF ? 8 : 1; }

// Tile shapes that are instantiated: accumulators (NACC * RPW * MT * NTW
// 16x16 tiles) within 16, RPW up to 2 in 2D and 4 in 3D.
template <int D, int EPI, int MT, int NTW, int RPW>
constexpr bool tile_ok() {
  return ((EPI == EPI_RESID) ? 2 : 1) * RPW * MT * NTW <= 16 && RPW <= ((D == 2) ? 2 : 4);
}

// One block of the convolution: `vblk` is the block index inside this
// problem's grid (the batched wrapper maps the launch's blocks onto problems).
template <int D, bool BF, int MODE, int EPI, int MT, int NTW, int RPW>
__device__ __forceinline__ void mconv_body(const MArgs& A, const int vblk, const int slice) {
  const gptr<const float> __restrict__ x = to_global<const float>(A.x);
  const gptr<const unsigned char> wA = to_global<const unsigned char>(A.wA);
  const gptr<const unsigned char> wB = to_global<const unsigned char>(A.wB);
  const gptr<float> __restrict__ y = to_global<float>(A.y);
  const gptr<const float> __restrict__ r = to_global<const float>(A.r);
  const gptr<const float> __restrict__ feat = to_global<const float>(A.feat);
  const int cin = A.cin, cinp = A.cinp, cout = A.cout, ncols = A.ncols, nsteps = A.nsteps;
  const int npairs = A.npairs, tiles_x = A.tiles_x, tiles_y = A.tiles_y, tiles_z = A.tiles_z;
  const int kchunk = A.kchunk;
  const Dims in = A.in, out = A.out;
  using G = Geo<D, MODE, MT, RPW>;
  constexpr int KV = KVOF<BF>();
  constexpr int NACC = (EPI == EPI_RESID) ? 2 : 1;
  constexpr int ES = BF ? 2 : 4;
  extern __shared__ __align__(16) unsigned char smem[];
  const int stride = mfma_lds_stride(D, BF, cin, cinp);  // LDS node stride (elements)
  unsigned char* bsm = smem + (((size_t)G::NODES * stride * ES + 15) / 16) * 16;
  constexpr int BROW = NTW * 16 * KV;      // elements of one pair row in the chunk
  constexpr int V16 = BROW * ES / 16;      // 16-byte vectors per row

  const int ntiles = tiles_x * tiles_y * tiles_z;
  const int per = (ntiles + 7) / 8;
  const int tl = (vblk % 8) * per + vblk / 8;
  if (tl >= ntiles) return;
  const int tx = tl % tiles_x, ty = (tl / tiles_x) % tiles_y, tz = tl / (tiles_x * tiles_y);
  const int x0 = tx * G::TX, y0 = ty * G::TY, z0 = tz * G::TZ;
  const int col0 = slice * NTW * 16;
  // grids: 2D (n[0] rows, n[1] x), 3D (n[0] z, n[1] y, n[2] x)
  const int IX = (D == 2) ? in.n[1] : in.n[2], IY = (D == 2) ? in.n[0] : in.n[1];
  const int IZ = (D == 2) ? 1 : in.n[0];
  const int OX = (D == 2) ? out.n[1] : out.n[2], OY = (D == 2) ? out.n[0] : out.n[1];
  const int OZ = (D == 2) ? 1 : out.n[0];
  // origin of the staged tile in input coordinates
  int sx, sy, sz;
  if (MODE == CONV_S1) { sx = x0 - 1; sy = y0 - 1; sz = z0 - 1; }
  else if (MODE == CONV_S2) { sx = 2 * x0 - 1; sy = 2 * y0 - 1; sz = 2 * z0 - 1; }
  else { sx = x0; sy = y0; sz = z0; }
  if (D == 2) sz = 0;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;

  // Weight chunk [s0, s0 + ks): rows q in [4 s0, 4 (s0 + ks)), columns
  // [col0, col0 + 16 NTW), laid out in LDS as [a][4 ks rows][BROW] so that
  // 16-byte vector idx of the chunk sits at byte 16 idx.  A wave's 64
  // consecutive vectors are then one contiguous 1 KB run, which the direct
  // global-to-LDS load writes (lane l at base + 16 l) with no registers and
  // no wait in the issuing wave; the wave waits for its own copies (vmcnt)
  // before the barrier that publishes the chunk.
  auto wsrc = [&](int s0, int ks, int idx) {
    const int nrow = 4 * ks;
    const int a = idx / (nrow * V16), rem = idx % (nrow * V16);
    const int row = rem / V16, vv = rem % V16;
    return (a ? wB : wA) + (((size_t)(4 * s0 + row) * ncols + col0) * KV) * ES + (size_t)vv * 16;
  };
  auto wfetch = [&](int s0, int ks, unsigned char* dst) {
    const int total = NACC * 4 * ks * V16;
    for (int base = wave * 64; base < total; base += 256) {
      const int idx = base + lane;
      if (idx < total) lds_copy16(wsrc(s0, ks, idx), dst + (size_t)__builtin_amdgcn_readfirstlane(base) * 16);
    }
  };
  // Several chunks are double-buffered: chunk c sits in buffer c % 2, and
  // chunk c + 1 is copied into the other buffer while chunk c is consumed.
  // 3D float32: the B fragments come straight from the packed weights in
  // global memory (L2-resident), so nothing but the input tile is staged
  // and more blocks fit a CU; the first two groups of steps are requested
  // before the staging.  (2D float32, with short K loops on small grids, is
  // faster with the weights staged in LDS.)
  constexpr bool BG = !BF && D == 3;
  const size_t cbytes = (size_t)NACC * 4 * kchunk * BROW * ES;
  const int ks0 = nsteps < kchunk ? nsteps : kchunk;
  if constexpr (!BG) wfetch(0, ks0, bsm);
  constexpr int GS = 4;   // K steps per group of B loads (float32)
  // B register sets: group j sits in set j % NB and is requested NB groups
  // before its products, about 32 matrix products ahead whatever the tile
  // (an L2 round trip is longer than the 8 products of two one-row groups)
  constexpr int PERG = GS * MT * NTW * RPW * NACC;   // products per group
  constexpr int NB = !BG ? 1 : PERG >= 16 ? 2 : PERG >= 8 ? 4 : 8;
  static_assert(!BG || MFMA_PAD_STEPS >= (2 * NB - 2) * GS + 4, "look-ahead past the zero steps");
  float bq[NB][GS][NACC][NTW];   // unused unless BG
  // B fragments of the group of four steps s0 .. s0 + 3 (s0 a multiple of
  // 4), tile t: with the weights packed by step groups (mfma_bg_index) they
  // are one 16-byte vector per lane and tensor, at vector (s0 + lg) ncols +
  // col0 + 16 t + li.  Groups past the end read the zero steps stored after
  // the tensor and are never multiplied.
  const int blane = lg * ncols + col0 + li;
  auto loadB = [&](int s0, float (&b)[GS][NACC][NTW]) {
    static_assert(GS == 4, "one vector per lane holds a group");
    const gptr<const float4> wAf = (gptr<const float4>)wA + (size_t)s0 * ncols;
    const gptr<const float4> wBf = (gptr<const float4>)wB + (size_t)s0 * ncols;
#pragma unroll
    for (int aa = 0; aa < NACC; ++aa)
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        const float4 v = gld(aa ? wBf : wAf, (long long)(blane + t * 16));
        b[0][aa][t] = v.x;
        b[1][aa][t] = v.y;
        b[2][aa][t] = v.z;
        b[3][aa][t] = v.w;
      }
  };
  if constexpr (BG) {
#pragma unroll
    for (int b = 0; b < NB; ++b) loadB(b * GS, bq[b]);
  }

  // ---- stage the input tile: loads are issued in batches of SB per thread
  // before any LDS store, so a block waits for one memory latency per batch
  // (small tiles, used on small grids, take the whole tile in one batch)
  {
    constexpr int SB = (RPW * MT * NTW <= 2) ? (BG ? 16 : 12) : 8;
    const bool vec4 = (cin % 4) == 0;
    const int ng = cinp / 4;
    const int total = G::NODES * ng;
    // 3D float32 with whole groups of 4 channels: the batch's loads are
    // unconditional (an index outside the grid is clamped to 0 and the value
    // replaced by zero), so all of them are in flight at once, and the
    // (node, channel group) split takes a float reciprocal instead of an
    // integer division (exact: idx < 2^15)
    if (BG && vec4) {
      const float inv_ng = 1.0f / (float)ng;
      // element offset of the staged tile's origin (negative at the low
      // boundary: only ever added to an in-grid offset)
      const long long tile0 = (((long long)sz * IY + sy) * IX + sx) * cin;
      auto split = [&](int idx, int& node, int& c) {
        node = (int)(((float)idx + 0.5f) * inv_ng);
        c = (idx - node * ng) * 4;
      };
      for (int base = threadIdx.x; base < total; base += 256 * SB) {
        float4 t[SB];
        bool ok[SB];
#pragma unroll
        for (int k = 0; k < SB; ++k) {
          const int idx = base + k * 256;
          int node, c;
          split(idx, node, c);
          const int hz = node / (G::HX * G::HY), rem = node - hz * (G::HX * G::HY);
          const int hy = rem / G::HX, hx = rem - hy * G::HX;
          ok[k] = (idx < total) & ((unsigned)(sx + hx) < (unsigned)IX) & ((unsigned)(sy + hy) < (unsigned)IY) &
                  ((unsigned)(sz + hz) < (unsigned)IZ);
          const int rel = ((hz * IY + hy) * IX + hx) * cin + c;
          t[k] = gld((gptr<const float4>)(x + (ok[k] ? tile0 + rel : 0)), 0);
        }
#pragma unroll
        for (int k = 0; k < SB; ++k) {
          const int idx = base + k * 256;
          if (idx >= total) continue;
          int node, c;
          split(idx, node, c);
          const float4 v = ok[k] ? t[k] : make_float4(0.f, 0.f, 0.f, 0.f);
          float* sp = reinterpret_cast<float*>(smem) + (size_t)node * stride + c;
          sp[0] = v.x; sp[1] = v.y; sp[2] = v.z; sp[3] = v.w;
        }
      }
    } else if (BG && cin == 2) {
      // the C = 2 finest level (one group of 4 channels per node, 2 real):
      // one unconditional 8-byte load per node, zero-selected, stored as the
      // node's two floats (stride 2); the four floats after the last node
      // are zero (read by the padding channels' K lanes of that node)
      if (threadIdx.x < 4) reinterpret_cast<float*>(smem)[(size_t)G::NODES * 2 + threadIdx.x] = 0.f;
      const long long tile0 = (((long long)sz * IY + sy) * IX + sx) * 2;
      for (int base = threadIdx.x; base < total; base += 256 * SB) {
        float2 t[SB];
        bool ok[SB];
#pragma unroll
        for (int k = 0; k < SB; ++k) {
          const int node = base + k * 256;
          const int hz = node / (G::HX * G::HY), rem = node - hz * (G::HX * G::HY);
          const int hy = rem / G::HX, hx = rem - hy * G::HX;
          ok[k] = (node < total) & ((unsigned)(sx + hx) < (unsigned)IX) & ((unsigned)(sy + hy) < (unsigned)IY) &
                  ((unsigned)(sz + hz) < (unsigned)IZ);
          const int rel = ((hz * IY + hy) * IX + hx) * 2;
          t[k] = gld((gptr<const float2>)(x + (ok[k] ? tile0 + rel : 0)), 0);
        }
#pragma unroll
        for (int k = 0; k < SB; ++k) {
          const int node = base + k * 256;
          if (node >= total) continue;
          *reinterpret_cast<float2*>(reinterpret_cast<float*>(smem) + (size_t)node * 2) =
              make_float2(ok[k] ? t[k].x : 0.f, ok[k] ? t[k].y : 0.f);
        }
      }
    } else
    for (int base = threadIdx.x; base < total; base += 256 * SB) {
      float4 v[SB];
#pragma unroll
      for (int k = 0; k < SB; ++k) {
        v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
        const int idx = base + k * 256;
        if (idx >= total) continue;
        const int node = idx / ng, c = (idx % ng) * 4;
        const int hx = node % G::HX, hy = (node / G::HX) % G::HY, hz = node / (G::HX * G::HY);
        const int gx = sx + hx, gy = sy + hy, gz = sz + hz;
        if (gx >= 0 && gx < IX && gy >= 0 && gy < IY && gz >= 0 && gz < IZ && c < cin) {
          const long long g = (((long long)gz * IY + gy) * IX + gx) * cin;
          if (vec4) {
            v[k] = gld((gptr<const float4>)(x + g + c), 0);
          } else {
            v[k].x = x[g + c];
            if (c + 1 < cin) v[k].y = x[g + c + 1];
            if (c + 2 < cin) v[k].z = x[g + c + 2];
            if (c + 3 < cin) v[k].w = x[g + c + 3];
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
          const unsigned lo = (unsigned)f2bf(v[k].x) | ((unsigned)f2bf(v[k].y) << 16);
          const unsigned hi = (unsigned)f2bf(v[k].z) | ((unsigned)f2bf(v[k].w) << 16);
          *reinterpret_cast<uint2*>(reinterpret_cast<u16*>(smem) + (size_t)node * stride + c) = make_uint2(lo, hi);
        } else {
          float* s = reinterpret_cast<float*>(smem) + (size_t)node * stride + c;
          s[0] = v[k].x; s[1] = v[k].y; s[2] = v[k].z; s[3] = v[k].w;
        }
      }
    }
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's weight copies are in LDS
  __syncthreads();                                   // tile and first weight chunk published

  // output offsets and epilogue operands of every accumulator element; for
  // small tiles, and in 3D float32 wherever they take at most 16 registers
  // (more would cost a wave per SIMD), the operands are fetched here, so
  // their latency overlaps the K loop instead of following it
  constexpr bool PREF = RPW * MT * NTW <= 2 || (BG && RPW * MT * NTW * NACC <= 4);
  auto out_off = [&](int i, int m, int t, int rr) -> long long {
    const int rho = wave + 4 * i;
    const int gy = y0 + rho % G::TY, gz = z0 + rho / G::TY;
    const int col = col0 + t * 16 + li;
    const int gx = x0 + m * 16 + 4 * lg + rr;
    if (MODE == CONV_T2) {
      // column = class * cout + c; class bits: x fastest
      const int cls = col / cout, c = col - cls * cout;
      const int ax = cls & 1, ay = (cls >> 1) & 1, az = (D == 3) ? ((cls >> 2) & 1) : 0;
      const int fx = 2 * gx + ax, fy = 2 * gy + ay, fz = (D == 3) ? 2 * gz + az : 0;
      if (cls < (1 << D) && fx < OX && fy < OY && fz < OZ)
        return (((long long)fz * OY + fy) * OX + fx) * cout + c;
    } else {
      if (col < cout && gx < OX && gy < OY && gz < OZ)
        return (((long long)gz * OY + gy) * OX + gx) * cout + col;
    }
    return -1;
  };
  float pe0[PREF ? RPW : 1][PREF ? MT : 1][PREF ? NTW : 1][4];
  float pe1[PREF ? RPW : 1][PREF ? MT : 1][PREF ? NTW : 1][4];
  if constexpr (PREF && EPI != EPI_SET) {
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NTW; ++t)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            const long long o = out_off(i, m, t, rr);
            pe0[i][m][t][rr] = 0.f;
            pe1[i][m][t][rr] = 0.f;
            if (o >= 0) {
              if (EPI == EPI_ADD) pe0[i][m][t][rr] = y[o];
              else if (EPI == EPI_MUL) pe0[i][m][t][rr] = feat[o];
              else if (EPI == EPI_RESID) { pe0[i][m][t][rr] = r[o]; pe1[i][m][t][rr] = feat[o]; }
            }
          }
  }

  floatx4 acc[NACC][RPW][MT][NTW];
#pragma unroll
  for (int a = 0; a < NACC; ++a)
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NTW; ++t) acc[a][i][m][t] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int cpv = cinp / KV;
  const int KS = kchunk;
  // LDS element offset of tap (0, 0, 0) for each (row, m) of this lane: the
  // staged node of tap (dz, dy, dx) is this base plus (dz HY + dy) HX + dx
  // in every mode
  int abase[RPW][MT];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int rho = wave + 4 * i;
    const int wy = rho % G::TY, wz = rho / G::TY;
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      const int ox = m * 16 + li;   // output x inside the tile
      const int f = (MODE == CONV_S2) ? 2 : 1;
      abase[i][m] = ((f * wz * G::HY + f * wy) * G::HX + f * ox) * stride;
    }
  }
  // Small tiles (used on small grids, where a block's latency is the
  // launch's) and every float32 tile (one fragment is one register there)
  // read the fragments of step ss + 1 before the products of step ss are
  // issued (two register sets), so LDS latency overlaps the matrix cores;
  // larger bf16 tiles keep one set, for occupancy.  Every accumulator takes
  // the steps in order.  Steps are loaded in order, so the pair walk
  // advances once per load.
  constexpr bool PIPE = PREF || !BF;
  PairWalk pw;
  pw.init(lg, cpv, npairs);
  typedef typename std::conditional<BF, bf16x8, float>::type Frag;
  auto mma = [&](const Frag (&bf)[NACC][NTW], const Frag (&af)[RPW][MT]) {
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NTW; ++t)
#pragma unroll
          for (int a = 0; a < NACC; ++a) {
            if constexpr (BF) acc[a][i][m][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i][m], bf[a][t], acc[a][i][m][t], 0, 0, 0);
            else acc[a][i][m][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][m], bf[a][t], acc[a][i][m][t], 0, 0, 0);
          }
  };
  if constexpr (BG) {
    // float32: B fragments from global memory in groups of GS steps, two
    // register sets: group g sits in set g % 2, and group g + 2 is loaded
    // into that set as soon as group g has been multiplied, so each load has
    // two groups of products to land (the first two are issued before the
    // input tile is staged).  A fragments come from the staged tile, one
    // step ahead.  No barrier inside the K loop.
    // float32 packs one input channel per K lane group and pads the
    // channels to a multiple of 4, so the four pairs of a step are four
    // consecutive channels of ONE tap: the tap and its staged offset are
    // the same in every lane and advance as scalars (same pairs, same
    // order as the pair walk).
    if (cinp % 16 == 0) {
      // channels in whole groups of 16: the four steps of a group are four
      // channel quads of ONE tap, so the walker advances once per group and
      // the group's A fragments sit at fixed offsets (0, 4, 8, 12) from its
      // base; a group's fragments are read one group ahead (two register
      // sets).  nsteps is a multiple of 4 here.
      int q_cb = 0, q_dx = 0, q_dy = 0, q_toff = 0, q_k = 0;
      const int ngroups = nsteps / GS;
      auto loadAq = [&](Frag (&af)[GS][RPW][MT]) {
        const int aoff = q_toff * stride + q_cb + lg;
#pragma unroll
        for (int g = 0; g < GS; ++g)
#pragma unroll
          for (int i = 0; i < RPW; ++i)
#pragma unroll
            for (int m = 0; m < MT; ++m)
              af[g][i][m] = reinterpret_cast<const float*>(smem)[abase[i][m] + aoff + 4 * g];
        // (stops at the last group, so the look-ahead stays inside the tile)
        if (++q_k < ngroups) {
          q_cb += 4 * GS;
          if (q_cb == cinp) {
            q_cb = 0;
            ++q_dx;
            ++q_toff;
            if (q_dx == G::W) {
              q_dx = 0;
              ++q_dy;
              q_toff += G::HX - G::W;
              if (q_dy == G::W) { q_dy = 0; q_toff += (G::HY - G::W) * G::HX; }
            }
          }
        }
      };
      Frag aq[2][GS][RPW][MT];
      loadAq(aq[0]);
      for (int s0 = 0; s0 < nsteps; s0 += NB * GS) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          loadAq(aq[(b + 1) & 1]);
          if (b == 0 || s0 + b * GS < nsteps) {
#pragma unroll
            for (int g = 0; g < GS; ++g) mma(bq[b][g], aq[b & 1][g]);
          }
          loadB(s0 + (b + NB) * GS, bq[b]);
        }
      }
    } else {
      int s_cb = 0, s_dx = 0, s_dy = 0, s_toff = 0, s_k = 0;
      // fragments of the walker's step, then one step on; the walker stops at
      // the last step, so the look-ahead reads past it stay inside the tile
      auto loadA = [&](Frag (&af)[RPW][MT]) {
        const int aoff = s_toff * stride + s_cb + lg;
  #pragma unroll
        for (int i = 0; i < RPW; ++i)
  #pragma unroll
          for (int m = 0; m < MT; ++m) af[i][m] = reinterpret_cast<const float*>(smem)[abase[i][m] + aoff];
        if (++s_k < nsteps) {
          s_cb += 4;
          if (s_cb == cinp) {
            s_cb = 0;
            ++s_dx;
            ++s_toff;
            if (s_dx == G::W) {
              s_dx = 0;
              ++s_dy;
              s_toff += G::HX - G::W;
              if (s_dy == G::W) { s_dy = 0; s_toff += (G::HY - G::W) * G::HX; }
            }
          }
        }
      };
      // A fragments two steps ahead in four register sets (set = step mod 4,
      // a compile-time index inside a group): the fragments of step s + 2 are
      // requested before the products of step s are issued, so two steps of
      // products cover their LDS latency
      Frag aset[GS][RPW][MT];
      loadA(aset[0]);
      loadA(aset[1]);
      auto group = [&](int s0, const float (&b)[GS][NACC][NTW]) {
  #pragma unroll
        for (int g = 0; g < GS; ++g) {
          loadA(aset[(g + 2) % GS]);
          if (s0 + g < nsteps) mma(b[g], aset[g]);
        }
      };
      // the look-ahead loads are unconditional (past the end they read the
      // zero steps stored after the tensor, or the tile's last step): every
      // path through the loop then has the same loads in flight, so the
      // compiler's counter waits stay exact instead of assuming a skipped load
      for (int s0 = 0; s0 < nsteps; s0 += NB * GS) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          if (b == 0 || s0 + b * GS < nsteps) group(s0 + b * GS, bq[b]);
          loadB(s0 + (b + NB) * GS, bq[b]);
        }
      }
    }
  } else {
    for (int s0 = 0, chunk = 0; s0 < nsteps; s0 += KS, ++chunk) {
      const int ks = (nsteps - s0) < KS ? (nsteps - s0) : KS;
      const unsigned char* cur = bsm + (chunk & 1) * cbytes;
      const bool more = s0 + KS < nsteps;
      // the other buffer was released by the barrier that ended the previous
      // chunk, so the next chunk's copy can start before this one is used
      if (more) wfetch(s0 + KS, (nsteps - s0 - KS) < KS ? (nsteps - s0 - KS) : KS, bsm + ((chunk + 1) & 1) * cbytes);
      auto load = [&](int ss, Frag (&bf)[NACC][NTW], Frag (&af)[RPW][MT]) {
        int tap, cb;
        pw.take(tap, cb);
        int dz = 0, dy, dx;
        if (D == 2) { dy = tap / G::W; dx = tap % G::W; }
        else { dz = tap / (G::W * G::W); dy = (tap / G::W) % G::W; dx = tap % G::W; }
        const int aoff = ((dz * G::HY + dy) * G::HX + dx) * stride + cb * KV;
  #pragma unroll
        for (int a = 0; a < NACC; ++a)
  #pragma unroll
          for (int t = 0; t < NTW; ++t) {
            const size_t o = ((size_t)a * 4 * ks + 4 * ss + lg) * BROW + (t * 16 + li) * KV;
            if constexpr (BF) bf[a][t] = *reinterpret_cast<const bf16x8*>(reinterpret_cast<const u16*>(cur) + o);
            else bf[a][t] = reinterpret_cast<const float*>(cur)[o];
          }
  #pragma unroll
        for (int i = 0; i < RPW; ++i)
  #pragma unroll
          for (int m = 0; m < MT; ++m) {
            if constexpr (BF) af[i][m] = *reinterpret_cast<const bf16x8*>(reinterpret_cast<const u16*>(smem) + abase[i][m] + aoff);
            else af[i][m] = reinterpret_cast<const float*>(smem)[abase[i][m] + aoff];
          }
      };
      Frag b0[NACC][NTW], a0[RPW][MT];
      if constexpr (PIPE) {
        Frag b1[NACC][NTW], a1[RPW][MT];
        load(0, b0, a0);
        int ss = 0;
        for (; ss + 1 < ks; ss += 2) {
          load(ss + 1, b1, a1);
          mma(b0, a0);
          if (ss + 2 < ks) load(ss + 2, b0, a0);
          mma(b1, a1);
        }
        if (ss < ks) mma(b0, a0);
      } else {
        for (int ss = 0; ss < ks; ++ss) {
          load(ss, b0, a0);
          mma(b0, a0);
        }
      }
      if (more) {
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's copies of the next chunk
        __syncthreads();                                   // next chunk published, this one released
      }
    }

  }

  // ---- epilogue: per (row, m) the operands of all its outputs are loaded
  // first (unless prefetched; in 3D float32 as unconditional loads with a
  // clamped index, so that they are all in flight together), then combined
  // and stored
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
#pragma unroll
    for (int m = 0; m < MT; ++m) {
      long long o[NTW][4];
      float e0[NTW][4], e1[NTW][4];
#pragma unroll
      for (int t = 0; t < NTW; ++t)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          o[t][rr] = out_off(i, m, t, rr);
          if constexpr (PREF) {
            e0[t][rr] = pe0[PREF ? i : 0][PREF ? m : 0][PREF ? t : 0][rr];
            e1[t][rr] = pe1[PREF ? i : 0][PREF ? m : 0][PREF ? t : 0][rr];
          } else if constexpr (BG) {
            const long long oc = o[t][rr] >= 0 ? o[t][rr] : 0;
            e0[t][rr] = 0.f;
            e1[t][rr] = 0.f;
            if (EPI == EPI_ADD) e0[t][rr] = y[oc];
            else if (EPI == EPI_MUL) e0[t][rr] = feat[oc];
            else if (EPI == EPI_RESID) { e0[t][rr] = r[oc]; e1[t][rr] = feat[oc]; }
          } else {
            e0[t][rr] = 0.f;
            e1[t][rr] = 0.f;
            if (o[t][rr] >= 0) {
              if (EPI == EPI_ADD) e0[t][rr] = y[o[t][rr]];
              else if (EPI == EPI_MUL) e0[t][rr] = feat[o[t][rr]];
              else if (EPI == EPI_RESID) { e0[t][rr] = r[o[t][rr]]; e1[t][rr] = feat[o[t][rr]]; }
            }
          }
        }
#pragma unroll
      for (int t = 0; t < NTW; ++t)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          if (o[t][rr] < 0) continue;
          float v = acc[0][i][m][t][rr];
          if (EPI == EPI_ADD) v = e0[t][rr] + v;
          else if (EPI == EPI_MUL) v = e0[t][rr] * v;
          else if (EPI == EPI_RESID) v = e0[t][rr] - v - e1[t][rr] * acc[NACC - 1][i][m][t][rr];
          y[o[t][rr]] = v;
        }
    }
  }
}

// One problem: the blocks of all column slices share one grid dimension,
// slices interleaved in runs of 8 (block b of run q is tile 8 q + b % 8 of
// slice (b / 8) % nslices), so the slices of a tile are dispatched together
// and to the same XCD (b mod 8) instead of one whole slice after another.
template <int D, bool BF, int MODE, int EPI, int MT, int NTW, int RPW>
__global__ __launch_bounds__(256) void mconv_kernel(MArgs A, int nslices) {
  const int run = blockIdx.x / (8 * nslices), rem = blockIdx.x % (8 * nslices);
  mconv_body<D, BF, MODE, EPI, MT, NTW, RPW>(A, run * 8 + rem % 8, rem / 8);
}

// Batched form: one launch for several problems; pre[p] is the first block of
// problem p (pre[np] = total blocks), tab[p] its arguments.
template <int D, bool BF, int MODE, int EPI, int MT, int NTW, int RPW>
__global__ __launch_bounds__(256) void mconv_kernel_batched(const MArgs* __restrict__ tab,
                                                            const int* __restrict__ pre, int np,
                                                            const int* __restrict__ frozen,
                                                            const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const MArgs A = tab[batch_entry(row, np, p)];
  mconv_body<D, BF, MODE, EPI, MT, NTW, RPW>(A, blockIdx.x - pre[p], blockIdx.y);
}

template <int D, bool BF, int MODE, int EPI, int MT, int NTW, int RPW>
hipError_t run(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  if constexpr (!tile_ok<D, EPI, MT, NTW, RPW>()) {
    return hipErrorInvalidValue;
  } else {
    const int nslices = a.ncols / (16 * NTW);
    const size_t lds = mfma_lds_bytes(a.dim, a.bf16, a.mode, a.mt, a.ntw, a.rpw, a.cin, a.cinp, a.epi, a.kchunk,
                                      a.nsteps);
    if (b) {
      hipLaunchKernelGGL((mconv_kernel_batched<D, BF, MODE, EPI, MT, NTW, RPW>), dim3(b->total, nslices),
                         dim3(256), lds, s, (const MArgs*)b->tab, b->pre, b->np, b->frozen, b->row);
    } else {
      int nblk;
      const MArgs A = mfma_args(a, &nblk);
      hipLaunchKernelGGL((mconv_kernel<D, BF, MODE, EPI, MT, NTW, RPW>), dim3(nblk * nslices), dim3(256),
                         lds, s, A, nslices);
    }
    return hipGetLastError();
  }
}

template <int D, bool BF, int MODE, int EPI, int MT, int NTW>
hipError_t by_rpw(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  switch (a.rpw) {
    case 1: return run<D, BF, MODE, EPI, MT, NTW, 1>(a, b, s);
    case 2: return run<D, BF, MODE, EPI, MT, NTW, 2>(a, b, s);
    case 4: return run<D, BF, MODE, EPI, MT, NTW, 4>(a, b, s);
  }
  return hipErrorInvalidValue;
}

template <int D, bool BF, int MODE, int EPI, int MT>
hipError_t by_ntw(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  switch (a.ntw) {
    case 1: return by_rpw<D, BF, MODE, EPI, MT, 1>(a, b, s);
    case 2: return by_rpw<D, BF, MODE, EPI, MT, 2>(a, b, s);
    case 4: return by_rpw<D, BF, MODE, EPI, MT, 4>(a, b, s);
  }
  return hipErrorInvalidValue;
}

template <int D, bool BF, int MODE, int EPI>
hipError_t by_mt(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  switch (a.mt) {
    case 1: return by_ntw<D, BF, MODE, EPI, 1>(a, b, s);
    case 2: return by_ntw<D, BF, MODE, EPI, 2>(a, b, s);
    case 4: return by_ntw<D, BF, MODE, EPI, 4>(a, b, s);
  }
  return hipErrorInvalidValue;
}

template <int D, bool BF>
hipError_t by_mode_s1(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  if (a.mode != CONV_S1) return hipErrorInvalidValue;
  switch (a.epi) {
    case EPI_SET: return by_mt<D, BF, CONV_S1, EPI_SET>(a, b, s);
    case EPI_ADD: return by_mt<D, BF, CONV_S1, EPI_ADD>(a, b, s);
    case EPI_MUL: return by_mt<D, BF, CONV_S1, EPI_MUL>(a, b, s);
    case EPI_RESID: return by_mt<D, BF, CONV_S1, EPI_RESID>(a, b, s);
  }
  return hipErrorInvalidValue;
}

template <int D, bool BF>
hipError_t by_mode_st(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  if (a.mode == CONV_S2 && a.epi == EPI_SET) return by_mt<D, BF, CONV_S2, EPI_SET>(a, b, s);
  if (a.mode == CONV_T2 && a.epi == EPI_ADD) return by_mt<D, BF, CONV_T2, EPI_ADD>(a, b, s);
  return hipErrorInvalidValue;
}

}  // namespace

}  // namespace mcmg

// One instantiation unit: NAME runs dimension D, precision BF, mode group
// GROUP (s1: stride-1 convolutions; st: restriction and prolongation).
#define MCONV_UNIT(NAME, D, BF, GROUP)                                                   \
  namespace mcmg {                                                                        \
  hipError_t NAME(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {              \
    return by_mode_##GROUP<D, BF>(a, b, s);                                               \
  }                                                                                       \
  }
