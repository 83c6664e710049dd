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
// column and a chunk of ZC planes and walks it plane by plane, keeping the
// last planes of e (halo 3 in y and x), t (halo 2) and u (halo 1) in LDS
// rings.  Each plane of t and u is then computed once per block (a cube
// tile with a halo of 3 recomputes about four times the work), and only the
// in-plane halos are shared with neighbouring blocks.  The tap loop runs
// over dz at run time with the 9 in-plane taps unrolled, so at most one
// plane's weights are live (the fully unrolled 27-tap form spills).
#include <type_traits>

#include "internal.h"

namespace mcmg {

namespace {

template <int D> struct G1;
template <> struct G1<2> { static constexpr int TZ = 1, TY = 8, TX = 64; };
// 3D z-streaming tile: TY x TX nodes per plane, ZC planes per block
struct G3 { static constexpr int TY = 8, TX = 64, ZC = 32; };

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

// Ring slot of plane `pl` (pl >= -4 R) in a ring of R planes.
__device__ __forceinline__ int ring(int pl, int R) { return (pl + 4 * R) % R; }

template <int VAR>
__device__ __forceinline__ void l1z_body(const L1Args& A, const L1Weights* __restrict__ wp,
                                         const int vblk) {
  constexpr int TY = G3::TY, TX = G3::TX, ZC = G3::ZC;
  constexpr int H = (VAR == L1_RESID) ? 1 : 3;           // y-x halo of the staged e
  constexpr int EY = TY + 2 * H, EX = TX + 2 * H, NE = EY * EX;
  constexpr int NER = (VAR == L1_STEP) ? 4 : 3;          // e ring (STEP keeps e of the output plane)
  constexpr int TYt = TY + 4, TXt = TX + 4, NT = TYt * TXt;
  constexpr int UY = TY + 2, UX = TX + 2, NU = UY * UX;
  constexpr int NO = TY * TX;
  constexpr int PE = (NE + NTH - 1) / NTH, PT = (NT + NTH - 1) / NTH;
  constexpr int PU = (NU + NTH - 1) / NTH, PO = (NO + NTH - 1) / NTH;
  __shared__ float2 se[(VAR == L1_FIRST) ? 1 : NER * NE];
  __shared__ float2 st[(VAR == L1_RESID) ? 1 : 3 * NT];
  __shared__ float2 su[(VAR == L1_RESID) ? 1 : 3 * NU];

  const gptr<const float2> __restrict__ e = to_global<const float2>(A.e);
  const gptr<float2> __restrict__ eo = to_global<float2>(A.eo);
  const gptr<const float2> __restrict__ r = to_global<const float2>(A.r);
  const gptr<const float2> __restrict__ a = to_global<const float2>(A.a);
  const gptr<const float2> __restrict__ s = to_global<const float2>(A.s);
  const gptr<const L1Weights> wg = to_global<const L1Weights>(wp);
  const int NZ = A.n.n[0], NY = A.n.n[1], NX = A.n.n[2];
  const int ntiles = A.tiles_x * A.tiles_y * A.tiles_z;
  const int per = (ntiles + 7) / 8;
  const int tl = (vblk % 8) * per + vblk / 8;   // XCD-contiguous bands
  if (tl >= ntiles) return;
  const int x0 = (tl % A.tiles_x) * TX, y0 = ((tl / A.tiles_x) % A.tiles_y) * TY;
  const int zb = (tl / (A.tiles_x * A.tiles_y)) * ZC;
  const int ze = min(zb + ZC, NZ);
  auto inside = [&](int z, int y, int x) {
    return x >= 0 && x < NX && y >= 0 && y < NY && z >= 0 && z < NZ;
  };
  auto gidx = [&](int z, int y, int x) { return ((long long)z * NY + y) * NX + x; };
  const float2 zero = make_float2(0.f, 0.f);

  // e plane k on the e box (zero outside the grid)
  auto load_e = [&](int k) {
    float2 v[PE];
#pragma unroll
    for (int j = 0; j < PE; ++j) {
      const int i = threadIdx.x + j * NTH;
      const int y = i / EX, x = i % EX;
      const int gy = y0 - H + y, gx = x0 - H + x;
      v[j] = ldz(e, gidx(k, gy, gx), i < NE && inside(k, gy, gx));
    }
    float2* dst = se + ring(k, NER) * NE;
#pragma unroll
    for (int j = 0; j < PE; ++j) {
      const int i = threadIdx.x + j * NTH;
      if (i < NE) dst[i] = v[j];
    }
  };
  // acc += (X * src)[point] over the 27 taps, src planes q-1, q, q+1 in a ring
  // (2 x 2 channel block X of the weight set `off` = W, KA, KS or Wsm).
  auto conv2 = [&](const float2* ring_base, int R, int plane_elems, int q, int pitch,
                   gptr<const float> Xw, const int* base, float* c0, float* c1, auto npts) {
    constexpr int NP = decltype(npts)::value;
#pragma unroll 1
    for (int dz = 0; dz < 3; ++dz) {
      const float2* P = ring_base + ring(q - 1 + dz, R) * plane_elems;
      const gptr<const float> w = Xw + dz * 9;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int to = (t / 3 - 1) * pitch + (t % 3 - 1);
        const float a00 = w[t], a01 = w[27 + t], a10 = w[54 + t], a11 = w[81 + t];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const float2 v = P[base[k] + to];
          c0[k] = fmaf(a00, v.x, fmaf(a01, v.y, c0[k]));
          c1[k] = fmaf(a10, v.x, fmaf(a11, v.y, c1[k]));
        }
      }
    }
  };
  // as conv2 for two weight sets X (into c0, c1) and Y (into d0, d1) that read
  // each staged value once; every accumulator sums its taps in conv2's order
  auto conv2pair = [&](const float2* ring_base, int R, int plane_elems, int q, int pitch,
                       gptr<const float> Xw, gptr<const float> Yw, const int* base, float* c0, float* c1,
                       float* d0, float* d1, auto npts) {
    constexpr int NP = decltype(npts)::value;
#pragma unroll 1
    for (int dz = 0; dz < 3; ++dz) {
      const float2* P = ring_base + ring(q - 1 + dz, R) * plane_elems;
      const gptr<const float> w = Xw + dz * 9;
      const gptr<const float> y = Yw + dz * 9;
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        const int to = (t / 3 - 1) * pitch + (t % 3 - 1);
        const float a00 = w[t], a01 = w[27 + t], a10 = w[54 + t], a11 = w[81 + t];
        const float b00 = y[t], b01 = y[27 + t], b10 = y[54 + t], b11 = y[81 + t];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const float2 v = P[base[k] + to];
          c0[k] = fmaf(a00, v.x, fmaf(a01, v.y, c0[k]));
          c1[k] = fmaf(a10, v.x, fmaf(a11, v.y, c1[k]));
          d0[k] = fmaf(b00, v.x, fmaf(b01, v.y, d0[k]));
          d1[k] = fmaf(b10, v.x, fmaf(b11, v.y, d1[k]));
        }
      }
    }
  };
  // t plane q on the t box (halo 2): t = r - W*e - a (.) (KA*e); FIRST: t = r
  auto make_t = [&](int q) {
    float2 rv[PT], av[PT];
    int eb[PT];
    bool ok[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int i = threadIdx.x + k * NTH;
      const int y = i / TXt, x = i % TXt;
      const int gy = y0 - 2 + y, gx = x0 - 2 + x;
      ok[k] = i < NT && inside(q, gy, gx);
      rv[k] = ldz(r, gidx(q, gy, gx), ok[k]);
      av[k] = (VAR != L1_FIRST) ? ldz(a, gidx(q, gy, gx), ok[k]) : zero;
      eb[k] = (i < NT) ? (y + H - 2) * EX + (x + H - 2) : EX + 1;
    }
    float w0[PT], w1[PT], k0[PT], k1[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) w0[k] = w1[k] = k0[k] = k1[k] = 0.f;
    if (VAR != L1_FIRST)
      conv2pair(se, NER, NE, q, EX, &wg->W[0][0][0], &wg->KA[0][0][0], eb, w0, w1, k0, k1,
                std::integral_constant<int, PT>());
    float2* dst = st + ring(q, 3) * NT;
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int i = threadIdx.x + k * NTH;
      if (i < NT)
        dst[i] = ok[k] ? make_float2(rv[k].x - w0[k] - av[k].x * k0[k], rv[k].y - w1[k] - av[k].y * k1[k])
                       : zero;
    }
  };
  // u plane p on the u box (halo 1): u = s (.) (KS * t)
  auto make_u = [&](int p) {
    float2 sv[PU];
    int tb[PU];
    bool ok[PU];
#pragma unroll
    for (int k = 0; k < PU; ++k) {
      const int i = threadIdx.x + k * NTH;
      const int y = i / UX, x = i % UX;
      const int gy = y0 - 1 + y, gx = x0 - 1 + x;
      ok[k] = i < NU && inside(p, gy, gx);
      sv[k] = ldz(s, gidx(p, gy, gx), ok[k]);
      tb[k] = (i < NU) ? (y + 1) * TXt + (x + 1) : TXt + 1;
    }
    float c0[PU], c1[PU];
#pragma unroll
    for (int k = 0; k < PU; ++k) c0[k] = c1[k] = 0.f;
    conv2(st, 3, NT, p, TXt, &wg->KS[0][0][0], tb, c0, c1, std::integral_constant<int, PU>());
    float2* dst = su + ring(p, 3) * NU;
#pragma unroll
    for (int k = 0; k < PU; ++k) {
      const int i = threadIdx.x + k * NTH;
      if (i < NU) dst[i] = ok[k] ? make_float2(sv[k].x * c0[k], sv[k].y * c1[k]) : zero;
    }
  };
  // output plane z: e' = e + Wsm * u
  auto make_out = [&](int z) {
    int ub[PO];
    bool ok[PO];
#pragma unroll
    for (int k = 0; k < PO; ++k) {
      const int i = threadIdx.x + k * NTH;
      const int y = i / TX, x = i % TX;
      ok[k] = i < NO && inside(z, y0 + y, x0 + x);
      ub[k] = (i < NO) ? (y + 1) * UX + (x + 1) : UX + 1;
    }
    float c0[PO], c1[PO];
#pragma unroll
    for (int k = 0; k < PO; ++k) c0[k] = c1[k] = 0.f;
    conv2(su, 3, NU, z, UX, &wg->Wsm[0][0][0], ub, c0, c1, std::integral_constant<int, PO>());
#pragma unroll
    for (int k = 0; k < PO; ++k) {
      if (!ok[k]) continue;
      const int i = threadIdx.x + k * NTH;
      const int y = i / TX, x = i % TX;
      float2 ev = zero;
      if (VAR == L1_STEP) ev = se[ring(z, NER) * NE + (y + H) * EX + (x + H)];
      gst(eo, gidx(z, y0 + y, x0 + x), make_float2(ev.x + c0[k], ev.y + c1[k]));
    }
  };

  if (VAR == L1_RESID) {
    // t = r - W*e - a (.) (KA*e) on the tile, e planes z-1..z+1 (halo 1)
    for (int k = zb - 1; k <= ze; ++k) {
      load_e(k);
      __syncthreads();
      const int z = k - 1;
      if (z >= zb) {
        int eb[PO];
        bool ok[PO];
        float2 rv[PO], av[PO];
#pragma unroll
        for (int j = 0; j < PO; ++j) {
          const int i = threadIdx.x + j * NTH;
          const int y = i / TX, x = i % TX;
          ok[j] = i < NO && inside(z, y0 + y, x0 + x);
          rv[j] = ldz(r, gidx(z, y0 + y, x0 + x), ok[j]);
          av[j] = ldz(a, gidx(z, y0 + y, x0 + x), ok[j]);
          eb[j] = (i < NO) ? (y + 1) * EX + (x + 1) : EX + 1;
        }
        float w0[PO], w1[PO], k0[PO], k1[PO];
#pragma unroll
        for (int j = 0; j < PO; ++j) w0[j] = w1[j] = k0[j] = k1[j] = 0.f;
        conv2pair(se, NER, NE, z, EX, &wg->W[0][0][0], &wg->KA[0][0][0], eb, w0, w1, k0, k1,
                  std::integral_constant<int, PO>());
#pragma unroll
        for (int j = 0; j < PO; ++j) {
          if (!ok[j]) continue;
          const int i = threadIdx.x + j * NTH;
          const int y = i / TX, x = i % TX;
          gst(eo, gidx(z, y0 + y, x0 + x), make_float2(rv[j].x - w0[j] - av[j].x * k0[j],
                                                       rv[j].y - w1[j] - av[j].y * k1[j]));
        }
      }
      __syncthreads();
    }
    return;
  }
  // STEP: at k, e plane k arrives, t plane k-1, u plane k-2, output plane k-3.
  // FIRST: t plane k (= r), u plane k-1, output plane k-2.
  constexpr int LAG = (VAR == L1_STEP) ? 1 : 0;
  for (int k = zb - 2 - LAG; k <= ze + 1 + LAG; ++k) {
    if (VAR == L1_STEP) {
      load_e(k);
      __syncthreads();
    }
    const int q = k - LAG, p = q - 1, z = q - 2;
    if (q >= zb - 2) make_t(q);
    __syncthreads();
    if (p >= zb - 1) make_u(p);
    __syncthreads();
    if (z >= zb) make_out(z);
    __syncthreads();
  }
}

template <int VAR>
__global__ __launch_bounds__(NTH) void l1z_kernel(L1Args A) {
  l1z_body<VAR>(A, A.wp, blockIdx.x);
}

template <int VAR>
__global__ __launch_bounds__(NTH) void l1z_kernel_batched(const L1Args* __restrict__ tab,
                                                          const int* __restrict__ pre, int np,
                                                          const int* __restrict__ frozen,
                                                          const int* __restrict__ row) {
  const int p = batch_find(pre, np, blockIdx.x);
  if (frozen && frozen[p]) return;
  const L1Args A = tab[batch_entry(row, np, p)];
  l1z_body<VAR>(A, A.wp, blockIdx.x - pre[p]);
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
      if (!l.wdev) return hipErrorInvalidValue;
      int nblk;
      const L1Args A = l1_args(l, l.wdev, &nblk);
      hipLaunchKernelGGL((l1z_kernel<VAR>), dim3(nblk), dim3(NTH), 0, s, A);
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

L1Args l1_args(const L1Launch& l, const L1Weights* wdev, int* nblk) {
  const int TX = l.dim == 2 ? G1<2>::TX : G3::TX, TY = l.dim == 2 ? G1<2>::TY : G3::TY;
  const int TZ = l.dim == 2 ? G1<2>::TZ : G3::ZC;
  const int NX = (l.dim == 2) ? l.n.n[1] : l.n.n[2], NY = (l.dim == 2) ? l.n.n[0] : l.n.n[1];
  const int NZ = (l.dim == 2) ? 1 : l.n.n[0];
  L1Args A;
  A.e = l.e; A.eo = l.eo; A.r = l.r; A.a = l.a; A.s = l.s; A.wp = wdev; A.n = l.n;
  A.tiles_x = (NX + TX - 1) / TX;
  A.tiles_y = (NY + TY - 1) / TY;
  A.tiles_z = (NZ + TZ - 1) / TZ;
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
