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
// Variants: FIRST (e = 0: u = s (.) (KS * r), e' = Wsm * u) and RESID
// (t = r - A e only, the input of the restriction).
#include "internal.h"

namespace mcmg {

namespace {

template <int D> struct G1;
template <> struct G1<2> { static constexpr int TZ = 1, TY = 32, TX = 64; };
template <> struct G1<3> { static constexpr int TZ = 2, TY = 4, TX = 32; };

template <int D, int VAR>
__global__ __launch_bounds__(256) void l1_kernel(const float2* __restrict__ e, float2* __restrict__ eo,
                                                 const float2* __restrict__ r, const float2* __restrict__ a,
                                                 const float2* __restrict__ s, L1Weights w, Dims n,
                                                 int tiles_x, int tiles_y, int tiles_z) {
  using G = G1<D>;
  constexpr int T = (D == 2) ? 9 : 27;
  constexpr int H = (VAR == L1_RESID) ? 1 : 3;           // halo of the staged e
  // staged boxes: e (halo H), t (halo 2), u (halo 1); 2D uses no z halo
  constexpr int HZ = (D == 2) ? 0 : 1;
  constexpr int EZ = G::TZ + 2 * H * HZ, EY = G::TY + 2 * H, EX = G::TX + 2 * H;
  constexpr int TZt = G::TZ + 4 * HZ, TYt = G::TY + 4, TXt = G::TX + 4;
  constexpr int UZ = G::TZ + 2 * HZ, UY = G::TY + 2, UX = G::TX + 2;
  __shared__ float2 se[(VAR == L1_FIRST) ? 1 : EZ * EY * EX];
  __shared__ float2 st[(VAR == L1_RESID) ? 1 : TZt * TYt * TXt];
  __shared__ float2 su[(VAR == L1_RESID) ? 1 : UZ * UY * UX];

  const int NX = (D == 2) ? n.n[1] : n.n[2], NY = (D == 2) ? n.n[0] : n.n[1];
  const int NZ = (D == 2) ? 1 : n.n[0];
  const int ntiles = tiles_x * tiles_y * tiles_z;
  const int per = (ntiles + 7) / 8;
  const int tl = (blockIdx.x % 8) * per + blockIdx.x / 8;   // XCD-contiguous bands
  if (tl >= ntiles) return;
  const int x0 = (tl % tiles_x) * G::TX, y0 = ((tl / tiles_x) % tiles_y) * G::TY;
  const int z0 = (tl / (tiles_x * tiles_y)) * G::TZ;
  auto inside = [&](int z, int y, int x) {
    return x >= 0 && x < NX && y >= 0 && y < NY && z >= 0 && z < NZ;
  };
  auto gidx = [&](int z, int y, int x) { return ((long long)z * NY + y) * NX + x; };
  auto off = [&](int t, int& dz, int& dy, int& dx) {
    if (D == 2) { dz = 0; dy = t / 3 - 1; dx = t % 3 - 1; }
    else { dz = t / 9 - 1; dy = (t / 3) % 3 - 1; dx = t % 3 - 1; }
  };

  // ---- stage e with halo H
  if (VAR != L1_FIRST) {
    const int oz = z0 - H * HZ, oy = y0 - H, ox = x0 - H;
    for (int i = threadIdx.x; i < EZ * EY * EX; i += 256) {
      const int x = i % EX, y = (i / EX) % EY, z = i / (EX * EY);
      const int gz = oz + z, gy = oy + y, gx = ox + x;
      se[i] = inside(gz, gy, gx) ? e[gidx(gz, gy, gx)] : make_float2(0.f, 0.f);
    }
    __syncthreads();
  }

  // ---- t = r - W*e - a (.) (KA*e) on the tile grown by 2 (RESID: the tile)
  if (VAR == L1_RESID) {
    for (int i = threadIdx.x; i < G::TZ * G::TY * G::TX; i += 256) {
      const int x = i % G::TX, y = (i / G::TX) % G::TY, z = i / (G::TX * G::TY);
      const int gz = z0 + z, gy = y0 + y, gx = x0 + x;
      if (!inside(gz, gy, gx)) continue;
      float w0 = 0.f, w1 = 0.f, k0 = 0.f, k1 = 0.f;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        int dz, dy, dx;
        off(t, dz, dy, dx);
        const float2 v = se[((z + 1 * HZ + dz) * EY + (y + 1 + dy)) * EX + (x + 1 + dx)];
        w0 += w.W[0][0][t] * v.x + w.W[0][1][t] * v.y;
        w1 += w.W[1][0][t] * v.x + w.W[1][1][t] * v.y;
        k0 += w.KA[0][0][t] * v.x + w.KA[0][1][t] * v.y;
        k1 += w.KA[1][0][t] * v.x + w.KA[1][1][t] * v.y;
      }
      const long long g = gidx(gz, gy, gx);
      const float2 rv = r[g], av = a[g];
      eo[g] = make_float2(rv.x - w0 - av.x * k0, rv.y - w1 - av.y * k1);
    }
    return;
  }

  {
    const int oz = z0 - 2 * HZ, oy = y0 - 2, ox = x0 - 2;
    for (int i = threadIdx.x; i < TZt * TYt * TXt; i += 256) {
      const int x = i % TXt, y = (i / TXt) % TYt, z = i / (TXt * TYt);
      const int gz = oz + z, gy = oy + y, gx = ox + x;
      float2 tv = make_float2(0.f, 0.f);
      if (inside(gz, gy, gx)) {
        const long long g = gidx(gz, gy, gx);
        const float2 rv = r[g];
        if (VAR == L1_FIRST) {
          tv = rv;
        } else {
          float w0 = 0.f, w1 = 0.f, k0 = 0.f, k1 = 0.f;
#pragma unroll
          for (int t = 0; t < T; ++t) {
            int dz, dy, dx;
            off(t, dz, dy, dx);
            const float2 v = se[((z + HZ + dz) * EY + (y + 1 + dy)) * EX + (x + 1 + dx)];
            w0 += w.W[0][0][t] * v.x + w.W[0][1][t] * v.y;
            w1 += w.W[1][0][t] * v.x + w.W[1][1][t] * v.y;
            k0 += w.KA[0][0][t] * v.x + w.KA[0][1][t] * v.y;
            k1 += w.KA[1][0][t] * v.x + w.KA[1][1][t] * v.y;
          }
          const float2 av = a[g];
          tv = make_float2(rv.x - w0 - av.x * k0, rv.y - w1 - av.y * k1);
        }
      }
      st[i] = tv;
    }
  }
  __syncthreads();

  // ---- u = s (.) (KS * t) on the tile grown by 1
  {
    const int oz = z0 - HZ, oy = y0 - 1, ox = x0 - 1;
    for (int i = threadIdx.x; i < UZ * UY * UX; i += 256) {
      const int x = i % UX, y = (i / UX) % UY, z = i / (UX * UY);
      const int gz = oz + z, gy = oy + y, gx = ox + x;
      float2 uv = make_float2(0.f, 0.f);
      if (inside(gz, gy, gx)) {
        float c0 = 0.f, c1 = 0.f;
#pragma unroll
        for (int t = 0; t < T; ++t) {
          int dz, dy, dx;
          off(t, dz, dy, dx);
          const float2 v = st[((z + HZ + dz) * TYt + (y + 1 + dy)) * TXt + (x + 1 + dx)];
          c0 += w.KS[0][0][t] * v.x + w.KS[0][1][t] * v.y;
          c1 += w.KS[1][0][t] * v.x + w.KS[1][1][t] * v.y;
        }
        const float2 sv = s[gidx(gz, gy, gx)];
        uv = make_float2(sv.x * c0, sv.y * c1);
      }
      su[i] = uv;
    }
  }
  __syncthreads();

  // ---- e' = e + Wsm * u on the tile
  for (int i = threadIdx.x; i < G::TZ * G::TY * G::TX; i += 256) {
    const int x = i % G::TX, y = (i / G::TX) % G::TY, z = i / (G::TX * G::TY);
    const int gz = z0 + z, gy = y0 + y, gx = x0 + x;
    if (!inside(gz, gy, gx)) continue;
    float c0 = 0.f, c1 = 0.f;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      int dz, dy, dx;
      off(t, dz, dy, dx);
      const float2 v = su[((z + HZ + dz) * UY + (y + 1 + dy)) * UX + (x + 1 + dx)];
      c0 += w.Wsm[0][0][t] * v.x + w.Wsm[0][1][t] * v.y;
      c1 += w.Wsm[1][0][t] * v.x + w.Wsm[1][1][t] * v.y;
    }
    float2 ev = make_float2(0.f, 0.f);
    if (VAR != L1_FIRST) ev = se[((z + H * HZ) * EY + (y + H)) * EX + (x + H)];
    eo[gidx(gz, gy, gx)] = make_float2(ev.x + c0, ev.y + c1);
  }
}

template <int D, int VAR>
hipError_t run(const L1Launch& l, hipStream_t s) {
  using G = G1<D>;
  const int NX = (D == 2) ? l.n.n[1] : l.n.n[2], NY = (D == 2) ? l.n.n[0] : l.n.n[1];
  const int NZ = (D == 2) ? 1 : l.n.n[0];
  const int tx = (NX + G::TX - 1) / G::TX, ty = (NY + G::TY - 1) / G::TY, tz = (NZ + G::TZ - 1) / G::TZ;
  const int nt = tx * ty * tz;
  hipLaunchKernelGGL((l1_kernel<D, VAR>), dim3(((nt + 7) / 8) * 8), dim3(256), 0, s,
                     (const float2*)l.e, (float2*)l.eo, (const float2*)l.r, (const float2*)l.a,
                     (const float2*)l.s, l.w, l.n, tx, ty, tz);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_level1(const L1Launch& l, hipStream_t s) {
  if (l.n.total == 0) return hipSuccess;
  if (l.dim == 2) {
    switch (l.var) {
      case L1_STEP: return run<2, L1_STEP>(l, s);
      case L1_FIRST: return run<2, L1_FIRST>(l, s);
      case L1_RESID: return run<2, L1_RESID>(l, s);
    }
  } else if (l.dim == 3) {
    switch (l.var) {
      case L1_STEP: return run<3, L1_STEP>(l, s);
      case L1_FIRST: return run<3, L1_FIRST>(l, s);
      case L1_RESID: return run<3, L1_RESID>(l, s);
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace mcmg
