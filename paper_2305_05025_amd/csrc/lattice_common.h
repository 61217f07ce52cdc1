// Device helpers shared by the lattice and atom kernels: population storage formats, the
// pull gather of a site's pre-collision values, the moments of Eqs. (2)-(3) and the
// external force density.
#pragma once

#include "lbmd_internal.h"

namespace lbmd {

// ---- storage formats --------------------------------------------------------------------
template <int ST>
struct Store;

template <>
struct Store<LB_STORE_F32> {
  using T = float;
  static __device__ __forceinline__ float ld(const T* p) { return *p; }
  static __device__ __forceinline__ void st(T* p, float v) { __builtin_nontemporal_store(v, p); }
};

template <>
struct Store<LB_STORE_F16> {
  using T = _Float16;
  static __device__ __forceinline__ float ld(const T* p) { return (float)*p; }
  // conversion to binary16 rounds to nearest even; subnormals are kept
  static __device__ __forceinline__ void st(T* p, float v) {
    __builtin_nontemporal_store((_Float16)v, p);
  }
};

template <>
struct Store<LB_STORE_BF16> {
  using T = uint16_t;
  static __device__ __forceinline__ float ld(const T* p) {
    return __uint_as_float((uint32_t)(*p) << 16);
  }
  static __device__ __forceinline__ void st(T* p, float v) {
    uint32_t u = __float_as_uint(v);
    uint16_t h;
    if ((u & 0x7fffffffu) > 0x7f800000u) {
      h = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    } else {
      u += 0x7fffu + ((u >> 16) & 1u);    // round to nearest, ties to even
      h = (uint16_t)(u >> 16);
    }
    __builtin_nontemporal_store(h, p);
  }
};

// ---- pull gather: pre-collision values at (x, y, z) -----------------------------------------
template <int ST>
__device__ __forceinline__ void gather(const typename Store<ST>::T* __restrict__ f, long plane,
                                       int x, int y, int z, int nx, int ny, int nz,
                                       float g[19]) {
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  const int nxy = nx * ny;
  const int X3[3] = {xm, x, xp};
  const int Y3[3] = {ym * nx, y * nx, yp * nx};
  const int Z3[3] = {zm * nxy, z * nxy, zp * nxy};
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int src = X3[1 - CX[i]] + Y3[1 - CY[i]] + Z3[1 - CZ[i]];
    g[i] = Store<ST>::ld(f + (size_t)i * plane + src);
  }
}

// ---- moments (Eqs. 2-3 in deviation form) --------------------------------------------------
__device__ __forceinline__ void moments(const float g[19], float& drho, float& jx, float& jy,
                                        float& jz) {
  drho = 0.f;
  jx = jy = jz = 0.f;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    drho += g[i];
    if (CX[i] == 1) jx += g[i];
    if (CX[i] == -1) jx -= g[i];
    if (CY[i] == 1) jy += g[i];
    if (CY[i] == -1) jy -= g[i];
    if (CZ[i] == 1) jz += g[i];
    if (CZ[i] == -1) jz -= g[i];
  }
}

template <int C>
__device__ __forceinline__ float cdot(float ax, float ay, float az, int cx, int cy, int cz) {
  float r = 0.f;
  if (cx == 1) r += ax;
  if (cx == -1) r -= ax;
  if (cy == 1) r += ay;
  if (cy == -1) r -= ay;
  if (cz == 1) r += az;
  if (cz == -1) r -= az;
  return r;
}

// ---- BGK + Guo collision in place; returns false on a non-finite moment ---------------------
__device__ __forceinline__ bool collide(float g[19], float Fx, float Fy, float Fz, float rho0,
                                        float omega, float pref) {
  float drho, jx, jy, jz;
  moments(g, drho, jx, jy, jz);
  const float rho = rho0 + drho;
  const float inv = 1.0f / rho;
  const float ux = (jx + 0.5f * Fx) * inv;
  const float uy = (jy + 0.5f * Fy) * inv;
  const float uz = (jz + 0.5f * Fz) * inv;
  const float uu = ux * ux + uy * uy + uz * uz;
  const float uF = ux * Fx + uy * Fy + uz * Fz;
  const float base = drho - 1.5f * rho * uu;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const float cu = cdot<0>(ux, uy, uz, CX[i], CY[i], CZ[i]);
    const float cF = cdot<0>(Fx, Fy, Fz, CX[i], CY[i], CZ[i]);
    const float geq = WQ[i] * (base + rho * (3.0f * cu + 4.5f * cu * cu));
    const float src = pref * WQ[i] * (3.0f * (cF - uF) + 9.0f * cu * cF);
    g[i] = g[i] - omega * (g[i] - geq) + src;
  }
  return __builtin_isfinite(drho + jx + jy + jz);
}

__device__ __forceinline__ void external_force(int bf_kind, const float* tab, const float* field,
                                               long plane, int s, int y, float& Fx, float& Fy,
                                               float& Fz) {
  Fx = Fy = Fz = 0.f;
  if (bf_kind == LB_BF_KOLMOGOROV || bf_kind == LB_BF_SIGN_SHEAR) {
    Fx = tab[y];
  } else if (bf_kind == LB_BF_FIELD) {
    Fx = field[s];
    Fy = field[plane + s];
    Fz = field[2 * plane + s];
  }
}

}  // namespace lbmd
