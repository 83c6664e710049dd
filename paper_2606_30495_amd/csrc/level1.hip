// Fused finest-level (C_1 = 2, the (Re, Im) channels) smoothing step of the
// V-cycle (Sec. 3.2):
//     t  = r - (W * e + a (.) (KA * e))       level operator residual
//     u  = s (.) (KS * t)                      feature-modulated smoother conv
//     e' = e + Wsm^(i) * u                     update
// in ONE pass over the grid.  A block stages e with a halo of 3 nodes in
// LDS, computes t on the tile grown by 2 and u on the tile grown by 1
// (recomputing the overlap instead of writing t and u to HBM), then writes
// e'.  Every convolution zero-pads its own input at the grid boundary, so t
// and u are set to zero outside the grid before they are convolved.
// Per node the pass streams e, r, a, s (8 bytes each) and writes e'
// (8 bytes): 40 B/node, the HBM-bound sweep of the V-cycle.  e' goes to a
// second buffer (neighbouring blocks still read e).
//
// Each phase runs tap-outermost: a thread owns a fixed set of points of the
// phase's box and keeps their accumulators in registers, so only one tap's
// 2 x 2 (x 2) weights are live at a time (wave-uniform scalars) and every
// tap costs one LDS read plus the FMAs per point.
//
// Variants: FIRST (e = 0: u = s (.) (KS * r), e' = Wsm * u) and RESID
// (t = r - A e only, the input of the restriction).
//
// 3D uses a z-streaming form instead of cube tiles: a block owns a TY x TX
// column and a chunk of planes (sized at launch) and walks it plane by
// plane, keeping planes of e (halo 3 in y and x), t (halo 2) and u (halo 1)
// in LDS.  Each plane of t and u is then computed once per block (a cube
// tile with a halo of 3 recomputes about four times the work), and only the
// in-plane halos are shared with neighbouring blocks.  Every staged plane is
// scattered once into the three output planes it feeds (see l1z_body); the
// in-plane taps run at run time, so at most one tap's (or one tap row's)
// weights are live (the fully unrolled 27-tap form spills).
#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace mcmg {

namespace {

template <int D> struct G1;
template <> struct G1<2> { static constexpr int TZ = 1, TY = 8, TX = 64; };
// 3D z-streaming tile: TY x TX nodes per plane; the planes per block (the
// z chunk) are chosen at launch.  9 x 54 fills the thread slots of every
// phase box well (t 13 x 58 in 3 x 256 slots, u 11 x 56 and e 15 x 60 in
// 3 and 4, the tile 9 x 54 in 2) and divides 216, 108 and 54 in x.
struct G3 { static constexpr int TY = 9, TX = 54; };

constexpr int NTH = 256;

// A weight read from LDS is the same in every lane: moving it to a scalar
// register keeps the vector registers for the points.
__device__ __forceinline__ float uni(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// p[i] if ok, else zero; the load is unconditional (index clamped to 0), so
// the value select does not become a load through a selected pointer
__device__ __forceinline__ float2 ldz(gptr<const float2> p, long long i, bool ok) {
  const float2 v = gld(p, ok ? i : 0);
  return ok ? v : make_float2(0.f, 0.f);
}

template <int D, int VAR, bool WL = false>
__device__ __forceinline__ void l1_body(const L1Args& A, const L1Weights& w, const int vblk) {
  static_assert(D == 2, "3D uses the z-streaming form");
  auto W_ = [](float v) { return WL ? uni(v) : v; };
  const gptr<const float2> __restrict__ e = to_global<const float2>(A.e);
  const gptr<float2> __restrict__ eo = to_global<float2>(A.eo);
  const gptr<const float2> __restrict__ r = to_global<const float2>(A.r);
  const gptr<const float2> __restrict__ a = to_global<const float2>(A.a);
  const gptr<const float2> __restrict__ s = to_global<const float2>(A.s);
  using G = G1<2>;
  constexpr int TY = G::TY, TX = G::TX;
  constexpr int H = (VAR == L1_RESID) ? 1 : 3;           // halo of the staged e
  constexpr int EY = TY + 2 * H, EX = TX + 2 * H, NE = EY * EX;
  constexpr int TG = (VAR == L1_RESID) ? 0 : 2;          // halo of the t box
  constexpr int TYt = TY + 2 * TG, TXt = TX + 2 * TG, NT = TYt * TXt;
  constexpr int UY = TY + 2, UX = TX + 2, NU = UY * UX;
  constexpr int NO = TY * TX;
  // points per thread in each phase: just enough slots for the phase's box
  // (every slot costs the full tap loop, used or not)
  constexpr int RT = (NT + NTH - 1) / NTH, RU = (NU + NTH - 1) / NTH, RO = (NO + NTH - 1) / NTH;
  constexpr int PE = (NE + NTH - 1) / NTH;                // staged e values per thread
  // LDS: `sa` holds e (halo H), then u (halo 1) once t exists; `sb` holds t.
  constexpr int NA = (VAR == L1_FIRST) ? NU : (VAR == L1_RESID ? NE : (NE > NU ? NE : NU));
  __shared__ float2 sa[NA];
  __shared__ float2 sb[(VAR == L1_RESID) ? 1 : NT];

  const int NX = A.n.n[1], NY = A.n.n[0];
  const int ntiles = A.tiles_x * A.tiles_y;
  const int per = (ntiles + 7) / 8;
  const int tl = (vblk % 8) * per + vblk / 8;   // XCD-contiguous bands
  if (tl >= ntiles) return;
  const int x0 = (tl % A.tiles_x) * TX, y0 = (tl / A.tiles_x) * TY;
  auto inside = [&](int y, int x) { return x >= 0 && x < NX && y >= 0 && y < NY; };
  auto gidx = [&](int y, int x) { return (long long)y * NX + x; };
  const float2 zero = make_float2(0.f, 0.f);

  // ---- every global operand of the block is requested up front, so the
  // block waits for one memory latency instead of one per phase: e with
  // halo H (staged in LDS), r and a on the t box, s on the u box, e on the
  // tile.  A thread owns the same points of each box throughout.
  float2 v[PE];
  if (VAR != L1_FIRST) {
#pragma unroll
    for (int k = 0; k < PE; ++k) {
      const int i = threadIdx.x + k * NTH;
      const int y = i / EX, x = i % EX;
      v[k] = ldz(e, gidx(y0 - H + y, x0 - H + x), i < NE && inside(y0 - H + y, x0 - H + x));
    }
  }
  float2 rv[RT], av[RT];
  int eb[RT];
  bool okt[RT];
#pragma unroll
  for (int k = 0; k < RT; ++k) {
    const int i = threadIdx.x + k * NTH;
    const int y = i / TXt, x = i % TXt;
    const int gy = y0 - TG + y, gx = x0 - TG + x;
    okt[k] = i < NT && inside(gy, gx);
    rv[k] = ldz(r, gidx(gy, gx), okt[k]);
    av[k] = (VAR != L1_FIRST) ? ldz(a, gidx(gy, gx), okt[k]) : zero;
    eb[k] = (i < NT) ? (y + H - TG) * EX + (x + H - TG) : EX + 1;
  }
  float2 sv[RU], ev[RO];
  int tb[RU], ub[RO];
  bool oku[RU], oko[RO];
  if (VAR != L1_RESID) {
#pragma unroll
    for (int k = 0; k < RU; ++k) {
      const int i = threadIdx.x + k * NTH;
      const int y = i / UX, x = i % UX;
      const int gy = y0 - 1 + y, gx = x0 - 1 + x;
      oku[k] = i < NU && inside(gy, gx);
      sv[k] = ldz(s, gidx(gy, gx), oku[k]);
      tb[k] = (i < NU) ? (y + 1) * TXt + (x + 1) : TXt + 1;
    }
#pragma unroll
    for (int k = 0; k < RO; ++k) {
      const int i = threadIdx.x + k * NTH;
      const int y = i / TX, x = i % TX;
      oko[k] = i < NO && inside(y0 + y, x0 + x);
      ub[k] = (i < NO) ? (y + 1) * UX + (x + 1) : UX + 1;
      ev[k] = (VAR != L1_FIRST) ? ldz(e, gidx(y0 + y, x0 + x), oko[k]) : zero;
    }
  }
  if (VAR != L1_FIRST) {
#pragma unroll
    for (int k = 0; k < PE; ++k) {
      const int i = threadIdx.x + k * NTH;
      if (i < NE) sa[i] = v[k];
    }
    __syncthreads();
  }

  // ---- t box: t = r - (W*e + a (.) (KA*e)) (FIRST: t = r; RESID: to memory)
  {
    float w0[RT], w1[RT], k0[RT], k1[RT];
#pragma unroll
    for (int k = 0; k < RT; ++k) w0[k] = w1[k] = k0[k] = k1[k] = 0.f;
    if (VAR != L1_FIRST) {
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int to = (t / 3 - 1) * EX + (t % 3 - 1);
        const float a00 = W_(w.W[0][0][t]), a01 = W_(w.W[0][1][t]), a10 = W_(w.W[1][0][t]), a11 = W_(w.W[1][1][t]);
        const float b00 = W_(w.KA[0][0][t]), b01 = W_(w.KA[0][1][t]), b10 = W_(w.KA[1][0][t]), b11 = W_(w.KA[1][1][t]);
#pragma unroll
        for (int k = 0; k < RT; ++k) {
          const float2 q = sa[eb[k] + to];
          w0[k] = fmaf(a00, q.x, fmaf(a01, q.y, w0[k]));
          w1[k] = fmaf(a10, q.x, fmaf(a11, q.y, w1[k]));
          k0[k] = fmaf(b00, q.x, fmaf(b01, q.y, k0[k]));
          k1[k] = fmaf(b10, q.x, fmaf(b11, q.y, k1[k]));
        }
      }
    }
#pragma unroll
    for (int k = 0; k < RT; ++k) {
      const int i = threadIdx.x + k * NTH;
      if (i >= NT) continue;
      const float2 tv = okt[k] ? make_float2(rv[k].x - w0[k] - av[k].x * k0[k], rv[k].y - w1[k] - av[k].y * k1[k])
                               : zero;
      if (VAR == L1_RESID) {
        if (okt[k]) gst(eo, gidx(y0 + i / TXt, x0 + i % TXt), tv);
      } else {
        sb[i] = tv;
      }
    }
  }
  if (VAR == L1_RESID) return;
  __syncthreads();

  // ---- u box: u = s (.) (KS * t), into the e storage (e is not read again)
  {
    float c0[RU], c1[RU];
#pragma unroll
    for (int k = 0; k < RU; ++k) c0[k] = c1[k] = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int to = (t / 3 - 1) * TXt + (t % 3 - 1);
      const float a00 = W_(w.KS[0][0][t]), a01 = W_(w.KS[0][1][t]), a10 = W_(w.KS[1][0][t]), a11 = W_(w.KS[1][1][t]);
#pragma unroll
      for (int k = 0; k < RU; ++k) {
        const float2 q = sb[tb[k] + to];
        c0[k] = fmaf(a00, q.x, fmaf(a01, q.y, c0[k]));
        c1[k] = fmaf(a10, q.x, fmaf(a11, q.y, c1[k]));
      }
    }
    // every thread has finished reading e from sa (barrier above) before u lands there
#pragma unroll
    for (int k = 0; k < RU; ++k) {
      const int i = threadIdx.x + k * NTH;
      if (i < NU) sa[i] = oku[k] ? make_float2(sv[k].x * c0[k], sv[k].y * c1[k]) : zero;
    }
  }
  __syncthreads();

  // ---- output tile: e' = e + Wsm * u
  {
    float c0[RO], c1[RO];
#pragma unroll
    for (int k = 0; k < RO; ++k) c0[k] = c1[k] = 0.f;
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      const int to = (t / 3 - 1) * UX + (t % 3 - 1);
      const float a00 = W_(w.Wsm[0][0][t]), a01 = W_(w.Wsm[0][1][t]), a10 = W_(w.Wsm[1][0][t]), a11 = W_(w.Wsm[1][1][t]);
#pragma unroll
      for (int k = 0; k < RO; ++k) {
        const float2 q = sa[ub[k] + to];
        c0[k] = fmaf(a00, q.x, fmaf(a01, q.y, c0[k]));
        c1[k] = fmaf(a10, q.x, fmaf(a11, q.y, c1[k]));
      }
    }
#pragma unroll
    for (int k = 0; k < RO; ++k) {
      if (!oko[k]) continue;
      const int i = threadIdx.x + k * NTH;
      gst(eo, gidx(y0 + i / TX, x0 + i % TX), make_float2(ev[k].x + c0[k], ev[k].y + c1[k]));
    }
  }
}

// Copy a weight set into LDS (all threads, then a barrier).
__device__ __forceinline__ void stage_weights(const L1Weights* __restrict__ src, L1Weights* dst) {
  constexpr int NW = sizeof(L1Weights) / sizeof(float);
  const gptr<const float> s = to_global<const float>(src);
  float* d = reinterpret_cast<float*>(dst);
  for (int i = threadIdx.x; i < NW; i += NTH) d[i] = s[i];
  __syncthreads();
}

// Element i of the tap-major 3D layout (see L1ZWeights) as an index into
// the [cout][cin][27 taps] layout of L1Weights.
__host__ __device__ inline int l1z_source(int i) {
  int tensor, t, dz, k;
  if (i < 216) {                     // WK[t][dz][8]: W block, then KA block
    t = i / 24; dz = (i / 8) % 3; k = i % 8;
    tensor = k < 4 ? 0 : 1;
    k &= 3;
  } else {                           // KS, Wsm: [t][dz][4]
    const int j = (i - 216) % 108;
    tensor = 2 + (i - 216) / 108;
    t = j / 12; dz = (j / 4) % 3; k = j % 4;
  }
  return tensor * 108 + k * 27 + dz * 9 + t;   // [cout][cin] = (k >> 1, k & 1)
}

__device__ __forceinline__ void stage_weights_z(const L1Weights* __restrict__ src, L1ZWeights* dst) {
  constexpr int NW = sizeof(L1ZWeights) / sizeof(float);
  const gptr<const float> s = to_global<const float>(src);
  float* d = reinterpret_cast<float*>(dst);
  for (int i = threadIdx.x; i < NW; i += NTH) d[i] = s[l1z_source(i)];
  __syncthreads();
}

// Ring slot of plane `pl` (pl >= -4 R) in a ring of R planes.
__device__ __forceinline__ int ring(int pl, int R) { return (pl + 4 * R) % R; }

// The z-march scatters every plane once: when plane k of a convolution's
// input is in LDS, each point reads its 9 in-plane taps there and adds them,
// with the dz = 2, 1, 0 weights, to the three outputs k - 1, k, k + 1 it
// feeds (accumulator slots 0, 1, 2 of the thread's points).  Output k - 1
// is then complete: it is finished, written, and the slots shift down by
// one.  An output still takes its contributions plane by plane (dz = 0, 1,
// 2) and tap by tap in row-major order, the order of a direct 27-tap sum,
// but every staged value is read from LDS once instead of three times.
// The weights come by value as a kernel argument (single problem: scalar
// loads from the argument segment) or staged in LDS (batched launches).
template <int VAR>
__device__ __forceinline__ void l1z_body(const L1Args& A, const L1ZWeights& wt, const int vblk) {
  constexpr int TY = G3::TY, TX = G3::TX;
  const int ZC = A.zc;
  constexpr bool STEP = VAR == L1_STEP, FIRST = VAR == L1_FIRST, RESID = VAR == L1_RESID;
  // e box (STEP: halo 3 around the tile; RESID: halo 1); FIRST has e = 0
  constexpr int H = RESID ? 1 : 3;
  constexpr int EY = TY + 2 * H, EX = TX + 2 * H, NE = EY * EX;
  // e planes held: k (being scattered) and k + 1 (being stored)
  constexpr int NER = 2;
  // t box (halo 2) for STEP / FIRST; RESID computes t on the tile
  constexpr int TG = RESID ? 0 : 2;
  constexpr int TYt = TY + 2 * TG, TXt = TX + 2 * TG, NT = TYt * TXt;
  constexpr int UY = TY + 2, UX = TX + 2, NU = UY * UX;
  constexpr int NO = TY * TX;
  constexpr int PE = (NE + NTH - 1) / NTH, PT = (NT + NTH - 1) / NTH;
  constexpr int PU = (NU + NTH - 1) / NTH, PO = (NO + NTH - 1) / NTH;
  // t plane (FIRST: r plane) on the t box, u plane on the u box; STEP keeps
  // two of each (one written, one read in the same iteration)
  constexpr int NTU = STEP ? 2 : 1;
  __shared__ float2 se[FIRST ? 1 : NER * NE];
  __shared__ float2 st[RESID ? 1 : NTU * NT];
  __shared__ float2 su[RESID ? 1 : NTU * NU];

  const gptr<const float2> __restrict__ e = to_global<const float2>(A.e);
  const gptr<float2> __restrict__ eo = to_global<float2>(A.eo);
  const gptr<const float2> __restrict__ r = to_global<const float2>(A.r);
  const gptr<const float2> __restrict__ a = to_global<const float2>(A.a);
  const gptr<const float2> __restrict__ s = to_global<const float2>(A.s);
  const L1ZWeights* wg = &wt;
  const int NZ = A.n.n[0], NY = A.n.n[1], NX = A.n.n[2];
  const int ntiles = A.tiles_x * A.tiles_y * A.tiles_z;
  const int per = (ntiles + 7) / 8;
  const int tl = (vblk % 8) * per + vblk / 8;   // XCD-contiguous bands
  if (tl >= ntiles) return;
  const int x0 = (tl % A.tiles_x) * TX, y0 = ((tl / A.tiles_x) % A.tiles_y) * TY;
  const int zb = (tl / (A.tiles_x * A.tiles_y)) * ZC;
  const int ze = min(zb + ZC, NZ);
  const int plane = NY * NX;
  const float2 zero = make_float2(0.f, 0.f);
  // A point's position is fixed for the whole march, so its in-plane grid
  // offset is computed once (-1 outside the grid or for an unused slot) and
  // a plane only adds a wave-uniform base: plane z of a tensor, clamped into
  // the grid (a plane outside it is only named by masked loads).
  auto poff = [&](bool used, int gy, int gx) {
    return (used && gy >= 0 && gy < NY && gx >= 0 && gx < NX) ? gy * NX + gx : -1;
  };
  auto at = [&](auto p, int z) { return p + (long long)min(max(z, 0), NZ - 1) * plane; };
  auto zin = [&](int z) { return z >= 0 && z < NZ; };
  // the point's value in plane pz, or zero outside the grid; the load is
  // unconditional (offset 0 when masked), so the select does not become a
  // load through a selected pointer
  auto ld = [&](gptr<const float2> pz, int off, bool zok) {
    const bool ok = zok && off >= 0;
    const float2 v = gld(pz, (long long)(unsigned)(ok ? off : 0));
    return ok ? v : zero;
  };

  // Scatter plane P (pitch = its box width) into the accumulators of the
  // outputs one behind (logical slot 0, dz = 2), level (slot 1, dz = 1) and
  // one ahead (slot 2, dz = 0) of it; logical slot q lives in register set
  // (q + R) % 3, R the phase of the march, so finishing an output renames
  // the sets instead of moving them.  T holds the tap-major weights: per
  // in-plane tap, per dz, the 2 x 2 channel block X (and, when PAIR, the
  // block Y of a second tensor read from the same values right after it),
  // so one tap's weights are one contiguous run.
  auto scatter = [&](auto rot, auto pair, const float2* P, int pitch, const float* T, const int* base,
                     auto& c0, auto& c1, auto& d0, auto& d1, auto npts) {
    constexpr int R = decltype(rot)::value;
    constexpr bool PAIR = decltype(pair)::value;
    constexpr int NP = decltype(npts)::value;
    constexpr int TS = PAIR ? 24 : 12;   // floats per in-plane tap
    // one tap's products on values v (weights wt of the tap)
    auto tap = [&](const float2 (&v)[NP], const float* wt) {
#pragma unroll
      for (int dz = 0; dz < 3; ++dz) {
        const int slot = (2 - dz + R) % 3;
        const float* w = wt + dz * (TS / 3);
        const float a00 = w[0], a01 = w[1], a10 = w[2], a11 = w[3];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          c0[slot][k] = fmaf(a00, v[k].x, fmaf(a01, v[k].y, c0[slot][k]));
          c1[slot][k] = fmaf(a10, v[k].x, fmaf(a11, v[k].y, c1[slot][k]));
        }
        if constexpr (PAIR) {
          const float b00 = w[4], b01 = w[5], b10 = w[6], b11 = w[7];
#pragma unroll
          for (int k = 0; k < NP; ++k) {
            d0[slot][k] = fmaf(b00, v[k].x, fmaf(b01, v[k].y, d0[slot][k]));
            d1[slot][k] = fmaf(b10, v[k].x, fmaf(b11, v[k].y, d1[slot][k]));
          }
        }
      }
    };
    // A row of taps per iteration where its values fit the registers (one
    // tensor: the u and output phases; two tensors with at most two points
    // per thread: the RESID form): the row's three taps' values are
    // requested together and waited for once, the weights of a row (36) or
    // of one tap (24) are live.  The STEP t phase (two tensors, three points
    // per thread) takes one tap per iteration.  Each accumulator takes the
    // taps in row-major order either way.
    constexpr bool ROWS = !PAIR || NP <= 2;
    if constexpr (ROWS) {
#pragma unroll 1
      for (int dy = 0; dy < 3; ++dy) {
        const int ro = (dy - 1) * pitch - 1;
        float2 v[3][NP];
#pragma unroll
        for (int dx = 0; dx < 3; ++dx)
#pragma unroll
          for (int k = 0; k < NP; ++k) v[dx][k] = P[base[k] + ro + dx];
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) tap(v[dx], T + (3 * dy + dx) * TS);
      }
    } else {
      // taps at run time, (dy, dx) row-major from (-1, -1)
      int to = -pitch - 1, dx = 0;
#pragma unroll 1
      for (int t = 0; t < 9; ++t) {
        float2 v[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) v[k] = P[base[k] + to];
        tap(v, T + t * TS);
        if (++dx == 3) {
          dx = 0;
          to += pitch - 2;
        } else {
          ++to;
        }
      }
    }
  };

  // logical slot 0 (set R) is finished: clear it, it becomes the next
  // phase's slot 2
  auto clear = [&](auto& c, auto rot) {
    constexpr int R = decltype(rot)::value;
    constexpr int NP = sizeof(c[0]) / sizeof(float);
#pragma unroll
    for (int k = 0; k < NP; ++k) c[R][k] = 0.f;
  };
  using std::integral_constant;

  // ---- per-thread points of each box, fixed for the whole march ----------
  // t box: LDS base of tap (0, 0) in the e box (RESID / STEP), grid offset
  int tb[PT], toff[PT];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int i = threadIdx.x + k * NTH;
    const int ty = i / TXt, tx = i % TXt;
    tb[k] = (i < NT) ? (ty + H - TG) * EX + (tx + H - TG) : EX + 1;
    toff[k] = poff(i < NT, y0 - TG + ty, x0 - TG + tx);
  }
  // u box: LDS base of tap (0, 0) in the t box, grid offset
  int ub[PU], uoff[PU];
#pragma unroll
  for (int k = 0; k < PU; ++k) {
    const int i = threadIdx.x + k * NTH;
    const int uy = i / UX, ux = i % UX;
    ub[k] = (i < NU) ? (uy + 1) * TXt + (ux + 1) : TXt + 1;
    uoff[k] = poff(i < NU, y0 - 1 + uy, x0 - 1 + ux);
  }
  // output tile: LDS base of tap (0, 0) in the u box, the point's e in the
  // e box, grid offset
  int ob[PO], oe[PO], ooff[PO];
#pragma unroll
  for (int k = 0; k < PO; ++k) {
    const int i = threadIdx.x + k * NTH;
    const int oy = i / TX, ox = i % TX;
    ob[k] = (i < NO) ? (oy + 1) * UX + (ox + 1) : UX + 1;
    oe[k] = (i < NO) ? (oy + H) * EX + (ox + H) : 0;
    ooff[k] = poff(i < NO, y0 + oy, x0 + ox);
  }
  // e box (STEP / RESID): grid offset
  constexpr int PEB = FIRST ? 1 : PE;
  int eoff[PEB];
#pragma unroll
  for (int k = 0; k < PEB; ++k) {
    const int i = threadIdx.x + k * NTH;
    eoff[k] = poff(i < NE, y0 - H + i / EX, x0 - H + i % EX);
  }

  // ---- the arriving plane's operands, loaded one iteration ahead ---------
  // STEP / RESID: e plane on the e box; FIRST: r plane on the t box
  constexpr int PIN = FIRST ? PT : PE;
  float2 vin[PIN];
  auto load_in = [&](int k) {
    const bool zok = zin(k);
#pragma unroll
    for (int j = 0; j < PIN; ++j) {
      if constexpr (FIRST) vin[j] = ld(at(r, k), toff[j], zok);
      else vin[j] = ld(at(e, k), eoff[j], zok);
    }
  };
  auto store_in = [&](int k) {
    float2* dst = FIRST ? st : se + ring(k, NER) * NE;
    constexpr int NB = FIRST ? NT : NE;
#pragma unroll
    for (int j = 0; j < PIN; ++j) {
      const int i = threadIdx.x + j * NTH;
      if (i < NB) dst[i] = vin[j];
    }
  };

  // ---- accumulators ---------------------------------------------------------
  float tw0[3][PT], tw1[3][PT], tk0[3][PT], tk1[3][PT];
  float uc0[3][PU], uc1[3][PU];
  float oc0[3][PO], oc1[3][PO];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
#pragma unroll
    for (int k = 0; k < PT; ++k) tw0[q][k] = tw1[q][k] = tk0[q][k] = tk1[q][k] = 0.f;
#pragma unroll
    for (int k = 0; k < PU; ++k) uc0[q][k] = uc1[q][k] = 0.f;
#pragma unroll
    for (int k = 0; k < PO; ++k) oc0[q][k] = oc1[q][k] = 0.f;
  }
  // operands of the outputs finished next: r, a of the t plane, s of the u
  // plane (loaded after their previous use, consumed one iteration later)
  float2 rv[PT], av[PT], sv[PU];
  auto load_ra = [&](int q) {
    const bool zok = zin(q);
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      rv[k] = ld(at(r, q), toff[k], zok);
      av[k] = ld(at(a, q), toff[k], zok);
    }
  };
  auto load_s = [&](int p) {
    const bool zok = zin(p);
#pragma unroll
    for (int k = 0; k < PU; ++k) sv[k] = ld(at(s, p), uoff[k], zok);
  };
  const integral_constant<int, 0> R0;
  const integral_constant<int, 1> R1;
  const integral_constant<int, 2> R2;

  if constexpr (RESID) {
    // plane k of e feeds t(k - 1), t(k), t(k + 1); t(k - 1) is written
    const int k0 = zb - 1, k1 = ze;
    load_in(k0);
    store_in(k0);
    load_ra(k0 - 1);
    auto iter = [&](int k, auto rot) {
      constexpr int R = decltype(rot)::value;
      if (k + 1 <= k1) load_in(k + 1);
      __syncthreads();                          // e(k) in LDS; e(k - 1)'s slot is free
      scatter(rot, integral_constant<bool, true>(), se + ring(k, NER) * NE, EX, &wg->WK[0][0][0], tb,
              tw0, tw1, tk0, tk1, integral_constant<int, PT>());
      const int q = k - 1;
      if (q >= zb) {
        const auto oq = at(eo, q);
#pragma unroll
        for (int j = 0; j < PT; ++j) {
          if (toff[j] >= 0)
            gst(oq, (long long)(unsigned)toff[j],
                make_float2(rv[j].x - tw0[R][j] - av[j].x * tk0[R][j],
                            rv[j].y - tw1[R][j] - av[j].y * tk1[R][j]));
        }
      }
      clear(tw0, rot); clear(tw1, rot); clear(tk0, rot); clear(tk1, rot);
      if (k + 1 <= k1) {
        load_ra(k);
        store_in(k + 1);                        // into the other slot of the pair
      }
    };
    for (int k = k0; k <= k1; k += 3) {
      iter(k, R0);
      if (k + 1 <= k1) iter(k + 1, R1);
      if (k + 2 <= k1) iter(k + 2, R2);
    }
    return;
  }

  if constexpr (STEP) {
    // One barrier per plane: the three scatters of an iteration are skewed
    // by one plane each, and the t and u planes are double-buffered.
    // Iteration k scatters e(k) into t and finishes t(k - 1) into st[k & 1];
    // scatters t(k - 2) (st[(k - 1) & 1], finished one iteration earlier)
    // into u and finishes u(k - 3) into su[k & 1]; scatters u(k - 4)
    // (su[(k - 1) & 1]) into the output and finishes out(k - 5), whose own e
    // each thread copied from the LDS ring when its plane was there and
    // carries in a five-deep register queue.  Every LDS read of an iteration
    // is of data written before its barrier, and every LDS buffer it writes
    // was last read before that barrier.  A scatter is skipped when all the outputs
    // it feeds lie outside the chunk's needs: t(zb - 2 .. ze + 1),
    // u(zb - 1 .. ze), out(zb .. ze - 1).
    const int k0 = zb - 3, k1 = ze + 4;
    // eq[q]: e at this thread's output points of plane k - 5 + q (entries of
    // planes before the chunk's first output are never used)
    float2 eq[5][PO];
#pragma unroll
    for (int q = 0; q < 5; ++q)
#pragma unroll
      for (int j = 0; j < PO; ++j) eq[q][j] = zero;
    load_in(k0);
    store_in(k0);
    load_ra(k0 - 1);
    load_s(k0 - 3);
    auto iter = [&](int k, auto rot) {
      constexpr int R = decltype(rot)::value;
      if (k + 1 <= ze + 2) load_in(k + 1);
      __syncthreads();                          // e(k), t(k - 2), u(k - 4) published
      // t(k - 1) = r - W e - a (.) (KA e), zero outside the grid
      if (k <= ze + 2)
        scatter(rot, integral_constant<bool, true>(), se + ring(k, NER) * NE, EX, &wg->WK[0][0][0], tb,
                tw0, tw1, tk0, tk1, integral_constant<int, PT>());
      {
        float2* stw = st + (k & 1) * NT;
        const bool qin = zin(k - 1);
#pragma unroll
        for (int j = 0; j < PT; ++j) {
          const int i = threadIdx.x + j * NTH;
          if (i < NT)
            stw[i] = (qin && toff[j] >= 0)
                         ? make_float2(rv[j].x - tw0[R][j] - av[j].x * tk0[R][j],
                                       rv[j].y - tw1[R][j] - av[j].y * tk1[R][j])
                         : zero;
        }
        clear(tw0, rot); clear(tw1, rot); clear(tk0, rot); clear(tk1, rot);
        load_ra(k);
      }
      // u(k - 3) = s (.) (KS * t), zero outside the grid
      if (k >= zb && k <= ze + 3)
        scatter(rot, integral_constant<bool, false>(), st + ((k - 1) & 1) * NT, TXt, &wg->KS[0][0][0],
                ub, uc0, uc1, uc0, uc1, integral_constant<int, PU>());
      {
        float2* suw = su + (k & 1) * NU;
        const bool pin = zin(k - 3);
#pragma unroll
        for (int j = 0; j < PU; ++j) {
          const int i = threadIdx.x + j * NTH;
          if (i < NU)
            suw[i] = (pin && uoff[j] >= 0) ? make_float2(sv[j].x * uc0[R][j], sv[j].y * uc1[R][j]) : zero;
        }
        clear(uc0, rot); clear(uc1, rot);
        load_s(k - 2);
      }
      // out(k - 5) = e + Wsm * u
      if (k >= zb + 3)
        scatter(rot, integral_constant<bool, false>(), su + ((k - 1) & 1) * NU, UX, &wg->Wsm[0][0][0],
                ob, oc0, oc1, oc0, oc1, integral_constant<int, PO>());
      {
        const int z = k - 5;
        if (z >= zb && z < ze) {
          const auto oz = at(eo, z);
#pragma unroll
          for (int j = 0; j < PO; ++j)
            if (ooff[j] >= 0)
              gst(oz, (long long)(unsigned)ooff[j], make_float2(eq[0][j].x + oc0[R][j], eq[0][j].y + oc1[R][j]));
        }
        clear(oc0, rot); clear(oc1, rot);
        // the queue moves on: e(k), in the ring this iteration, enters it
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int j = 0; j < PO; ++j) eq[q][j] = eq[q + 1][j];
#pragma unroll
        for (int j = 0; j < PO; ++j) eq[4][j] = se[ring(k, NER) * NE + oe[j]];
      }
      // e(k + 1) into the slot of e(k - 1), last read before the barrier
      if (k + 1 <= ze + 2) store_in(k + 1);
    };
    for (int k = k0; k <= k1; k += 3) {
      iter(k, R0);
      if (k + 1 <= k1) iter(k + 1, R1);
      if (k + 2 <= k1) iter(k + 2, R2);
    }
    return;
  }

  // FIRST (e = 0, t = r): plane k of r feeds u(k - 1 .. k + 1); u(k - 1)
  // feeds out(k - 2 .. k).
  const int k0 = zb - 2, k1 = ze + 1;
  load_in(k0);
  store_in(k0);
  load_s(k0 - 1);
  auto iter = [&](int k, auto rot) {
    constexpr int R = decltype(rot)::value;
    if (k + 1 <= k1) load_in(k + 1);
    __syncthreads();                            // input plane k published; su free
    // u(k - 1) = s (.) (KS * r), zero outside the grid
    {
      scatter(rot, integral_constant<bool, false>(), st, TXt, &wg->KS[0][0][0], ub, uc0, uc1, uc0, uc1,
              integral_constant<int, PU>());
      const int p = k - 1;
      const bool pin = zin(p);
#pragma unroll
      for (int j = 0; j < PU; ++j) {
        const int i = threadIdx.x + j * NTH;
        if (i < NU)
          su[i] = (pin && uoff[j] >= 0) ? make_float2(sv[j].x * uc0[R][j], sv[j].y * uc1[R][j]) : zero;
      }
      clear(uc0, rot); clear(uc1, rot);
      if (k + 1 <= k1) load_s(p + 1);
    }
    __syncthreads();                            // u(k - 1) published; the r plane consumed
    // out(k - 2) = Wsm * u.  u(p) feeds out(p - 1 .. p + 1), so it is
    // scattered only from p = zb - 1 on (the skipped planes' outputs are
    // discarded, and slots enter the window cleared).
    {
      if (k >= zb)
        scatter(rot, integral_constant<bool, false>(), su, UX, &wg->Wsm[0][0][0], ob, oc0, oc1, oc0,
                oc1, integral_constant<int, PO>());
      const int z = k - 2;
      if (z >= zb && z < ze) {
        const auto oz = at(eo, z);
#pragma unroll
        for (int j = 0; j < PO; ++j)
          if (ooff[j] >= 0)
            gst(oz, (long long)(unsigned)ooff[j], make_float2(oc0[R][j], oc1[R][j]));
      }
      clear(oc0, rot); clear(oc1, rot);
      // the next r plane: the current one was last read by this
      // iteration's u phase, finished at the barrier above
      if (k + 1 <= k1) store_in(k + 1);
    }
  };
  for (int k = k0; k <= k1; k += 3) {
    iter(k, R0);
    if (k + 1 <= k1) iter(k + 1, R1);
    if (k + 2 <= k1) iter(k + 2, R2);
  }
}

template <int VAR>
__global__ __launch_bounds__(NTH) void l1z_kernel(L1Args A, L1ZWeights w) {
  l1z_body<VAR>(A, w, blockIdx.x);
}

template <int VAR>
__global__ __launch_bounds__(NTH) void l1z_kernel_batched(const L1Args* __restrict__ tab,
                                                          const int* __restrict__ pre, int np,
                                                          const int* __restrict__ frozen,
                                                          const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const L1Args A = tab[batch_entry(row, np, p)];
  __shared__ L1ZWeights wsh;
  stage_weights_z(A.wp, &wsh);
  l1z_body<VAR>(A, wsh, blockIdx.x - pre[p]);
}

template <int D, int VAR>
__global__ __launch_bounds__(NTH) void l1_kernel(L1Args A, L1Weights w) {
  l1_body<D, VAR>(A, w, blockIdx.x);
}

// Batched form: tab[p] per problem (weights through A.wp), pre = block prefix.
template <int D, int VAR>
__global__ __launch_bounds__(NTH) void l1_kernel_batched(const L1Args* __restrict__ tab,
                                                         const int* __restrict__ pre, int np,
                                                         const int* __restrict__ frozen,
    const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const L1Args A = tab[batch_entry(row, np, p)];
  // the problem's weights (1.7 KB) are staged in LDS once per block and read
  // there with uniform addresses (through the table pointer they would be
  // vector loads held in registers)
  __shared__ L1Weights wsh;
  stage_weights(A.wp, &wsh);
  l1_body<D, VAR, true>(A, wsh, blockIdx.x - pre[p]);
}

template <int D, int VAR>
hipError_t run(const L1Launch& l, const BatchLaunch* b, hipStream_t s) {
  if constexpr (D == 3) {
    if (b) {
      hipLaunchKernelGGL((l1z_kernel_batched<VAR>), dim3(b->total), dim3(NTH), 0, s,
                         (const L1Args*)b->tab, b->pre, b->np, b->frozen, b->row);
    } else {
      int nblk;
      const L1Args A = l1_args(l, l.wdev, &nblk);
      L1ZWeights wz;
      const float* src = &l.w.W[0][0][0];
      float* dst = &wz.WK[0][0][0];
      for (int i = 0; i < (int)(sizeof(L1ZWeights) / sizeof(float)); ++i) dst[i] = src[l1z_source(i)];
      hipLaunchKernelGGL((l1z_kernel<VAR>), dim3(nblk), dim3(NTH), 0, s, A, wz);
    }
  } else {
    if (b) {
      hipLaunchKernelGGL((l1_kernel_batched<D, VAR>), dim3(b->total), dim3(NTH), 0, s,
                         (const L1Args*)b->tab, b->pre, b->np, b->frozen, b->row);
    } else {
      int nblk;
      const L1Args A = l1_args(l, nullptr, &nblk);
      hipLaunchKernelGGL((l1_kernel<D, VAR>), dim3(nblk), dim3(NTH), 0, s, A, l.w);
    }
  }
  return hipGetLastError();
}

hipError_t dispatch(const L1Launch& l, const BatchLaunch* b, hipStream_t s) {
  if (l.dim == 2) {
    switch (l.var) {
      case L1_STEP: return run<2, L1_STEP>(l, b, s);
      case L1_FIRST: return run<2, L1_FIRST>(l, b, s);
      case L1_RESID: return run<2, L1_RESID>(l, b, s);
    }
  } else if (l.dim == 3) {
    switch (l.var) {
      case L1_STEP: return run<3, L1_STEP>(l, b, s);
      case L1_FIRST: return run<3, L1_FIRST>(l, b, s);
      case L1_RESID: return run<3, L1_RESID>(l, b, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace

// Resident blocks per CU of the single-problem 3D kernel of a variant.
static int l1z_blocks_per_cu(int var) {
  static int cache[3] = {0, 0, 0};
  int& n = cache[var];
  if (n == 0) {
    int v = 0;
    hipError_t e = hipErrorInvalidValue;
    if (var == L1_STEP) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, l1z_kernel<L1_STEP>, NTH, 0);
    if (var == L1_FIRST) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, l1z_kernel<L1_FIRST>, NTH, 0);
    if (var == L1_RESID) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, l1z_kernel<L1_RESID>, NTH, 0);
    n = (e == hipSuccess && v > 0) ? v : 2;
  }
  return n;
}

L1Args l1_args(const L1Launch& l, const L1Weights* wdev, int* nblk, int nprob) {
  const int TX = l.dim == 2 ? G1<2>::TX : G3::TX, TY = l.dim == 2 ? G1<2>::TY : G3::TY;
  const int NX = (l.dim == 2) ? l.n.n[1] : l.n.n[2], NY = (l.dim == 2) ? l.n.n[0] : l.n.n[1];
  const int NZ = (l.dim == 2) ? 1 : l.n.n[0];
  L1Args A;
  A.e = l.e; A.eo = l.eo; A.r = l.r; A.a = l.a; A.s = l.s; A.wp = wdev; A.n = l.n;
  A.tiles_x = (NX + TX - 1) / TX;
  A.tiles_y = (NY + TY - 1) / TY;
  if (l.dim == 2) {
    A.zc = 1;
  } else {
    // the z chunk: as many chunks per column as fill one wave of resident
    // blocks (each chunk re-marches 6 planes of halo, so fewer, longer
    // chunks cost less once the chip is full), at least 4 planes
    const int cols = A.tiles_x * A.tiles_y;
    const int slots = l1z_blocks_per_cu(l.var) * device_cus() / std::max(1, nprob);
    const int chunks = std::max(1, slots / std::max(1, cols));
    A.zc = std::max(4, (NZ + chunks - 1) / chunks);
  }
  A.tiles_z = (NZ + A.zc - 1) / A.zc;
  const int nt = A.tiles_x * A.tiles_y * A.tiles_z;
  *nblk = ((nt + 7) / 8) * 8;
  return A;
}

hipError_t launch_level1(const L1Launch& l, hipStream_t s) {
  if (l.n.total == 0) return hipSuccess;
  return dispatch(l, nullptr, s);
}

hipError_t launch_level1_batched(int dim, int var, const BatchLaunch& b, hipStream_t s) {
  if (b.np == 0 || b.total == 0) return hipSuccess;
  L1Launch proto;
  proto.dim = dim;
  proto.var = var;
  return dispatch(proto, &b, s);
}

}  // namespace mcmg
