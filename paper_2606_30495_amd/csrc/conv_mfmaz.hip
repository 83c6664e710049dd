// z-marching form of the 3D float32 stride-1 matrix-core convolution for
// 12 -> 12 channels (the C = 12 level of the V-cycle, Sec. 3.2): the same
// implicit GEMM as conv_mfma.hip (K = 27 taps x 12 channels in 81 steps of
// v_mfma_f32_16x16x4f32, epilogues SET / ADD / MUL / RESID), organised so
// that a block's memory traffic overlaps its products.
//
// A block owns a 16 x 8 column of output nodes (x, y) and a chunk of zc
// output planes.  It copies the packed weights of its one or two tensors
// into LDS once (21 KB each), keeps the three input planes an output plane
// needs (z - 1, z, z + 1, with a halo of one node in x and y) in an LDS
// ring, and walks z: while plane z is computed, the next plane is already
// in registers (requested one plane earlier) and the epilogue operands of
// plane z are in flight.  The K loop reads only LDS, so the
// memory loads never wait behind weight loads, and it is fully unrolled:
// every tap's offset is a constant.  Each wave owns output rows y = w and
// y = w + 4 of the column (w = wave).  The summation order of every output
// is the one of conv_mfma.hip (K steps in order), so the two forms give the
// same bits.
#include <hip/hip_runtime.h>

#include "conv_mfma.h"
#include "internal.h"

namespace mcmg {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int ZTX = 16, ZTY = 8;               // output column of a block
constexpr int ZHX = ZTX + 2, ZHY = ZTY + 2;    // staged plane with its halo
constexpr int ZPN = ZHX * ZHY;                 // nodes of a staged plane
// LDS node stride: unpadded.  A fragment read has lane (li, lg) read
// channel 4 cq + lg of node li; with 12 floats per node the 16 nodes start
// on 16 distinct multiples of 4 banks, so the 64 lanes hit 64 distinct
// banks (a 13-float stride puts up to four lanes on one bank), and a
// channel quad is one 16-byte store when the plane is staged.
constexpr int ZC = 12, ZST = ZC;               // channels, LDS node stride
constexpr int ZPLANE = ZPN * ZST;              // floats of a ring slot
constexpr int ZSTEPS = 27 * ZC / 4;            // 81 K steps
constexpr int ZSTEPS4 = (ZSTEPS + 3) / 4 * 4;  // 84: whole runs of four steps
constexpr int ZBTEN = ZSTEPS4 * 4 * 16;        // floats of one packed tensor used
constexpr int ZPF = (ZPN * 3 + 255) / 256;     // float4 of a plane per thread

// Ring slots: the residual form (two weight tensors) keeps four, so the
// next plane is stored into the free slot before a plane's K loop and one
// barrier per plane suffices (80 KB: two blocks per CU); the one-tensor
// forms keep three (50 KB: three blocks per CU) and store it after the K
// loop, behind a second barrier.
constexpr int zslots(int epi) { return epi == EPI_RESID ? 4 : 3; }

template <int EPI>
__device__ __forceinline__ void mconvz_body(const MArgs& A, const int vblk) {
  constexpr int NACC = (EPI == EPI_RESID) ? 2 : 1;
  constexpr int NS = zslots(EPI);
  extern __shared__ __align__(16) float zsm[];
  float* ring = zsm;                    // [NS][ZPLANE]
  float* bs = zsm + NS * ZPLANE;        // [NACC][ZBTEN], the packed layout

  const gptr<const float> __restrict__ x = to_global<const float>(A.x);
  const gptr<float> __restrict__ y = to_global<float>(A.y);
  const gptr<const float> __restrict__ r = to_global<const float>(A.r);
  const gptr<const float> __restrict__ feat = to_global<const float>(A.feat);
  const int tiles_x = A.tiles_x, tiles_y = A.tiles_y, tiles_z = A.tiles_z, zc = A.zc;
  const int cout = A.cout;
  const int NZ = A.in.n[0], NY = A.in.n[1], NX = A.in.n[2];

  const int ntiles = tiles_x * tiles_y * tiles_z;
  const int per = (ntiles + 7) / 8;
  const int tl = (vblk % 8) * per + vblk / 8;   // XCD-contiguous bands
  if (tl >= ntiles) return;
  const int x0 = (tl % tiles_x) * ZTX, y0 = ((tl / tiles_x) % tiles_y) * ZTY;
  const int z0 = (tl / (tiles_x * tiles_y)) * zc;
  const int z1 = min(z0 + zc, NZ);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, lg = lane >> 4;

  // ---- planes: element idx of a plane is (node idx / 3, channel quad idx % 3)
  // of the staged 18 x 10 box; nodes outside the grid are zero.  A thread's
  // elements are the same in every plane, so their in-plane grid offsets are
  // computed once (-1 outside the grid); a plane adds a uniform base.  The
  // loads are unconditional (offset 0 when masked, value selected after).
  const long long pin = (long long)NY * NX * ZC;      // floats of an input plane
  int poff[ZPF];
#pragma unroll
  for (int k = 0; k < ZPF; ++k) {
    const int idx = threadIdx.x + 256 * k;
    const int node = idx / 3, c = (idx - 3 * node) * 4;
    const int hy = node / ZHX, hx = node - hy * ZHX;
    const int gx = x0 - 1 + hx, gy = y0 - 1 + hy;
    const bool ok = (idx < ZPN * 3) & ((unsigned)gx < (unsigned)NX) & ((unsigned)gy < (unsigned)NY);
    poff[k] = ok ? (gy * NX + gx) * ZC + c : -1;
  }
  float4 pf[ZPF];
  auto load_plane = [&](int z, float4 (&dst)[ZPF]) {
    const bool zok = (unsigned)z < (unsigned)NZ;
    const gptr<const float> xz = x + (zok ? z : 0) * pin;
#pragma unroll
    for (int k = 0; k < ZPF; ++k) {
      const bool ok = zok && poff[k] >= 0;
      const float4 v = gld((gptr<const float4>)(xz + (unsigned)(ok ? poff[k] : 0)), 0);
      dst[k] = ok ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto store_plane = [&](int z, const float4 (&src)[ZPF]) {
    float* slot = ring + ((z + NS) % NS) * ZPLANE;
#pragma unroll
    for (int k = 0; k < ZPF; ++k) {
      const int idx = threadIdx.x + 256 * k;
      if (idx < ZPN * 3) *reinterpret_cast<float4*>(slot + 4 * idx) = src[k];   // node idx / 3, channels 4 (idx % 3)
    }
  };
  // ---- prologue: the weights (the first ZSTEPS4 steps of each packed
  // tensor, as is) and the first three planes are requested together and
  // only then stored, so a block waits for one memory latency, not four;
  // the fourth plane stays in registers until plane z0 is done
  {
    const gptr<const float4> wa = (gptr<const float4>)A.wA;
    const gptr<const float4> wb = (gptr<const float4>)A.wB;
    constexpr int NV = ZBTEN / 4;
    constexpr int NW = (NACC * NV + 255) / 256;
    float4 wv[NW];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int i = min((int)threadIdx.x + 256 * k, NACC * NV - 1);
      wv[k] = gld(i < NV ? wa : wb, (long long)(i < NV ? i : i - NV));
    }
    float4 p0[ZPF], p1[ZPF], p2[ZPF];
    load_plane(z0 - 1, p0);
    load_plane(z0, p1);
    load_plane(z0 + 1, p2);
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      const int i = threadIdx.x + 256 * k;
      if (i < NACC * NV) *reinterpret_cast<float4*>(bs + 4 * i) = wv[k];
    }
    store_plane(z0 - 1, p0);
    store_plane(z0, p1);
    store_plane(z0 + 1, p2);
  }
  load_plane(z0 + 2, pf);

  // this lane's part of the A and B addresses; row i of the wave is y = w + 4 i
  int lbase[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) lbase[i] = ((wave + 4 * i) * ZHX + li) * ZST + lg;
  const int blane = (lg * 16 + li) * 4;

  // accumulator element (row i, r) is node (x0 + 4 lg + r, y0 + w + 4 i),
  // column li: its in-plane output offset is obase[i] + r cout; the row is
  // in the grid when rowok[i] (wave-uniform), the element when also
  // 4 lg + r < NX - x0 and li < cout
  const long long pout = (long long)NY * NX * cout;   // floats of an output plane
  int obase[2];
  bool rowok[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int gy = y0 + wave + 4 * i;
    rowok[i] = gy < NY;
    obase[i] = (min(gy, NY - 1) * NX + x0 + 4 * lg) * cout + li;
  }
  const int xlim = NX - x0 - 4 * lg;                  // element r is in the grid when r < xlim
  const bool colok = li < cout;
  auto elem_ok = [&](int i, int rr) { return rowok[i] && colok && rr < xlim; };

  for (int z = z0; z < z1; ++z) {
    __syncthreads();              // planes z - 1 .. z + 1 (and the weights) published
    if (NS == 4 && z + 1 < z1) {
      // plane z + 2 into the fourth slot (its plane z - 2 was last read
      // before the barrier above), the plane after it requested
      store_plane(z + 2, pf);
      if (z + 2 < z1) load_plane(z + 3, pf);
    }
    // epilogue operands of plane z: in flight during the K loop (the loads
    // are unconditional, offset 0 outside the grid)
    const long long zo = (long long)z * pout;
    float e0[2][4], e1[2][4];
    if constexpr (EPI != EPI_SET) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const unsigned oc = elem_ok(i, rr) ? (unsigned)(obase[i] + rr * cout) : 0u;
          if (EPI == EPI_ADD) e0[i][rr] = (y + zo)[oc];
          else if (EPI == EPI_MUL) e0[i][rr] = (feat + zo)[oc];
          else { e0[i][rr] = (r + zo)[oc]; e1[i][rr] = (feat + zo)[oc]; }
        }
    }
    const int sb[3] = {((z - 1 + NS) % NS) * ZPLANE, (z % NS) * ZPLANE, ((z + 1) % NS) * ZPLANE};
    floatx4 acc[NACC][2];
#pragma unroll
    for (int a = 0; a < NACC; ++a)
#pragma unroll
      for (int i = 0; i < 2; ++i) acc[a][i] = floatx4{0.f, 0.f, 0.f, 0.f};
    // K loop: step s = 3 tap + channel quad, tap = (dz, dy, dx) row-major.
    // Fully unrolled in groups of four steps; the A and B fragments of group
    // g + 1 are requested before the products of group g (two register
    // sets), so a group of products covers the LDS latency.
    constexpr int NG = ZSTEPS4 / 4;
    float av[2][4][2];
    float4 bv[2][NACC];
    auto loadg = [&](int g, int buf) {
#pragma unroll
      for (int a = 0; a < NACC; ++a)
        bv[buf][a] = *reinterpret_cast<const float4*>(bs + a * ZBTEN + g * 256 + blane);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int s = 4 * g + j;
        if (s >= ZSTEPS) continue;
        const int t = s / 3, cq = s - 3 * t;
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
        const int off = sb[dz] + (dy * ZHX + dx) * ZST + 4 * cq;
#pragma unroll
        for (int i = 0; i < 2; ++i) av[buf][j][i] = ring[lbase[i] + off];
      }
    };
    loadg(0, 0);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      if (g + 1 < NG) loadg(g + 1, (g + 1) & 1);
      // (keeps the scheduler from sinking those loads next to their uses)
      __builtin_amdgcn_sched_barrier(0);
      const int cur = g & 1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (4 * g + j >= ZSTEPS) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int a = 0; a < NACC; ++a) {
            const float b = j == 0 ? bv[cur][a].x : j == 1 ? bv[cur][a].y : j == 2 ? bv[cur][a].z : bv[cur][a].w;
            acc[a][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[cur][j][i], b, acc[a][i], 0, 0, 0);
          }
      }
    }
    // epilogue of plane z
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        float v = acc[0][i][rr];
        if (EPI == EPI_ADD) v = e0[i][rr] + v;
        else if (EPI == EPI_MUL) v = e0[i][rr] * v;
        else if (EPI == EPI_RESID) v = e0[i][rr] - v - e1[i][rr] * acc[NACC - 1][i][rr];
        if (elem_ok(i, rr)) (y + zo)[(unsigned)(obase[i] + rr * cout)] = v;
      }
    if (NS == 3 && z + 1 < z1) {
      __syncthreads();            // every wave is done with plane z - 1's slot
      store_plane(z + 2, pf);     // into that slot
      if (z + 2 < z1) load_plane(z + 3, pf);
    }
  }
}

template <int EPI>
__global__ __launch_bounds__(256) void mconvz_kernel(MArgs A) {
  mconvz_body<EPI>(A, blockIdx.x);
}

template <int EPI>
__global__ __launch_bounds__(256) void mconvz_kernel_batched(const MArgs* __restrict__ tab,
                                                             const int* __restrict__ pre, int np,
                                                             const int* __restrict__ frozen,
                                                             const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const MArgs A = tab[batch_entry(row, np, p)];
  mconvz_body<EPI>(A, blockIdx.x - pre[p]);
}

template <int EPI>
hipError_t runz(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  const size_t lds = mfmaz_lds_bytes(EPI);
  if (b) {
    hipLaunchKernelGGL((mconvz_kernel_batched<EPI>), dim3(b->total), dim3(256), lds, s,
                       (const MArgs*)b->tab, b->pre, b->np, b->frozen, b->row);
  } else {
    int nblk;
    const MArgs A = mfma_args(a, &nblk);
    hipLaunchKernelGGL((mconvz_kernel<EPI>), dim3(nblk), dim3(256), lds, s, A);
  }
  return hipGetLastError();
}

}  // namespace

size_t mfmaz_lds_bytes(int epi) {
  return (size_t)(zslots(epi) * ZPLANE + (epi == EPI_RESID ? 2 : 1) * ZBTEN) * sizeof(float);
}

bool mfmaz_ok(int dim, int bf16, int mode, int cin, int cout) {
  return dim == 3 && !bf16 && mode == CONV_S1 && cin == ZC && cout <= 16 && cout >= 1;
}

hipError_t launch_conv_mfmaz(const MfmaConv& a, const BatchLaunch* b, hipStream_t s) {
  if (!mfmaz_ok(a.dim, a.bf16, a.mode, a.cin, a.cout) || a.ncols != 16 || a.nsteps != ZSTEPS)
    return hipErrorInvalidValue;
  switch (a.epi) {
    case EPI_SET: return runz<EPI_SET>(a, b, s);
    case EPI_ADD: return runz<EPI_ADD>(a, b, s);
    case EPI_MUL: return runz<EPI_MUL>(a, b, s);
    case EPI_RESID: return runz<EPI_RESID>(a, b, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace mcmg
