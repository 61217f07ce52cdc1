// Device helpers shared by the lattice and atom kernels: population storage formats, the
// pull gather of a site's pre-collision values, the moments of Eqs. (2)-(3) and the
// external force density.
#pragma once

#include <type_traits>

#include "lbmd_internal.h"

namespace lbmd {

// ---- storage formats --------------------------------------------------------------------
template <int ST>
struct Store;

template <>
struct Store<LB_STORE_F32> {
  using T = float;
  template <class P>
  static __device__ __forceinline__ float ld(const P* p) { return *p; }
  template <class P>
  static __device__ __forceinline__ float ld_nt(const P* p) { return __builtin_nontemporal_load(p); }
  template <class P>
  static __device__ __forceinline__ void st(P* p, float v) { __builtin_nontemporal_store(v, p); }
};

template <>
struct Store<LB_STORE_F16> {
  using T = _Float16;
  template <class P>
  static __device__ __forceinline__ float ld(const P* p) { return (float)*p; }
  template <class P>
  static __device__ __forceinline__ float ld_nt(const P* p) { return (float)__builtin_nontemporal_load(p); }
  // conversion to binary16 rounds to nearest even; subnormals are kept
  template <class P>
  static __device__ __forceinline__ void st(P* p, float v) {
    __builtin_nontemporal_store((_Float16)v, p);
  }
};

template <>
struct Store<LB_STORE_BF16> {
  using T = uint16_t;
  template <class P>
  static __device__ __forceinline__ float ld(const P* p) {
    return __uint_as_float((uint32_t)(*p) << 16);
  }
  template <class P>
  static __device__ __forceinline__ float ld_nt(const P* p) {
    return __uint_as_float((uint32_t)__builtin_nontemporal_load(p) << 16);
  }
  // conversion by the hardware (v_cvt_pk_bf16_f32): round to nearest even, NaN stays NaN
  template <class P>
  static __device__ __forceinline__ void st(P* p, float v) {
    __builtin_nontemporal_store(__builtin_bit_cast(uint16_t, (__bf16)v), p);
  }
};

// ---- site coordinates ------------------------------------------------------------------
// s = x + nx (y + ny z) -> (x, y, z), by the invariant-divisor multiplications of FastDiv
__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv d) {
  return (__umulhi(n, d.m) + n) >> d.l;
}
__device__ __forceinline__ void site_xyz(int s, int nx, int ny, FastDiv dnx, FastDiv dny, int& x,
                                         int& y, int& z) {
  const uint32_t t = fdiv((uint32_t)s, dnx);
  const uint32_t zz = fdiv(t, dny);
  x = s - (int)t * nx;
  y = (int)t - (int)zz * ny;
  z = (int)zz;
}

// Element at byte offset `off` of population plane i, for lattices whose planes hold at
// most 4 GiB of sites.  The plane's base is uniform across the launch; the empty asm statement
// pins it to scalar registers as an opaque value, so every access takes the scalar-base +
// 32-bit-lane-offset form.  (Without it the compiler folds the shared lane offset of a site's
// Q stores into one 64-bit lane address and adds each plane's stride to it in 64-bit vector
// arithmetic.)
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* plane_at(T* f, int i, long plane,
                                                                       uint32_t off) {
  uint64_t b = reinterpret_cast<uint64_t>(f + (size_t)i * plane);
  asm("" : "+s"(b));
  return (__attribute__((address_space(1))) T*)(b + off);
}

// ---- pull gather: pre-collision values at (x, y, z) -----------------------------------------
// Q = 19 or 27 velocities (the default 19 is the D3Q19 set of Eq. 1).  `narrow`: the
// lattice's planes fit 32-bit byte offsets (uniform across the launch).  NT: the loads are
// non-temporal (the sweep reads every stored value exactly once, so keeping its lines in L2
// only displaces the data of the kernels that run beside it; gathers at scattered nodes,
// whose neighbouring rows share lines, keep the default).
template <int ST, int Q = 19, bool NT = false>
__device__ __forceinline__ void gather(const typename Store<ST>::T* __restrict__ f, long plane,
                                       int x, int y, int z, int nx, int ny, int nz, bool narrow,
                                       float g[Q]) {
  using T = typename Store<ST>::T;
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  const int nxy = nx * ny;
  if (narrow) {
    constexpr uint32_t E = sizeof(T);
    const uint32_t X3[3] = {E * xm, E * x, E * xp};
    const uint32_t Y3[3] = {E * nx * ym, E * nx * y, E * nx * yp};
    const uint32_t Z3[3] = {E * nxy * zm, E * nxy * z, E * nxy * zp};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const auto* p = plane_at(f, i, plane, X3[1 - CX[i]] + Y3[1 - CY[i]] + Z3[1 - CZ[i]]);
      g[i] = NT ? Store<ST>::ld_nt(p) : Store<ST>::ld(p);
    }
  } else {
    const int X3[3] = {xm, x, xp};
    const int Y3[3] = {ym * nx, y * nx, yp * nx};
    const int Z3[3] = {zm * nxy, z * nxy, zp * nxy};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int src = X3[1 - CX[i]] + Y3[1 - CY[i]] + Z3[1 - CZ[i]];
      const auto* p = f + (size_t)i * plane + src;
      g[i] = NT ? Store<ST>::ld_nt(p) : Store<ST>::ld(p);
    }
  }
}

// ---- moments (Eqs. 2-3 in deviation form) --------------------------------------------------
template <int Q = 19>
__device__ __forceinline__ void moments(const float g[Q], float& drho, float& jx, float& jy,
                                        float& jz) {
  drho = 0.f;
  jx = jy = jz = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
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
template <int Q = 19>
__device__ __forceinline__ bool collide(float g[Q], float Fx, float Fy, float Fz, float rho0,
                                        float omega, float pref) {
  float drho, jx, jy, jz;
  moments<Q>(g, drho, jx, jy, jz);
  const float rho = rho0 + drho;
  const float inv = 1.0f / rho;
  const float ux = (jx + 0.5f * Fx) * inv;
  const float uy = (jy + 0.5f * Fy) * inv;
  const float uz = (jz + 0.5f * Fz) * inv;
  const float uu = ux * ux + uy * uy + uz * uz;
  const float uF = ux * Fx + uy * Fy + uz * Fz;
  const float base = drho - 1.5f * rho * uu;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float cu = cdot<0>(ux, uy, uz, CX[i], CY[i], CZ[i]);
    const float cF = cdot<0>(Fx, Fy, Fz, CX[i], CY[i], CZ[i]);
    const float geq = wq<Q>(i) * (base + rho * (3.0f * cu + 4.5f * cu * cu));
    const float src = pref * wq<Q>(i) * (3.0f * (cF - uF) + 9.0f * cu * cF);
    g[i] = g[i] - omega * (g[i] - geq) + src;
  }
  return __builtin_isfinite(drho + jx + jy + jz);
}

// ---- thermal noise (fluctuating LB) -------------------------------------------------------
// The source term of Eq. 1 carries, besides the forces, Gaussian noise xi_i on the moments
// the collision does not conserve (Section 2.2).  xi_i = w_i A sum_{k=4..18} e_k(c_i) z_k /
// sqrt(b_k): e_k the orthogonal D3Q19 moment basis (density, momentum, stresses, kinetic
// modes), b_k = sum_i w_i e_k(c_i)^2, A = sqrt(3 rho kT (1 - (1 - omega)^2)) with rho the
// local density before the collision, z_k standard normals.  Each non-conserved mode then
// receives variance 3 rho kT b_k (1 - (1 - omega)^2), which keeps it at its equilibrium
// fluctuation under the relaxation factor 1 - omega; mass and momentum get none.
//
// On the D3Q27 lattice the basis is the products P_a(c_x) P_b(c_y) P_c(c_z) of the
// one-dimensional three-speed polynomials P_0 = 1, P_1 = c, P_2 = 3 c^2 - 1 (norms 1, 1/3, 2
// under the weights 2/3, 1/6, 1/6): density and momentum, then 23 non-conserved modes.
//
// Normals: Philox4x32-10 (a counter-based generator) keyed by the seed, counter (site, step
// low word, step high word, q) for q = 0..3 (D3Q19) or 0..5 (D3Q27); each 32-bit output w
// gives the uniform ((w >> 8) + 1/2) 2^-24, and pairs of uniforms give Box-Muller normals.

__device__ __forceinline__ void philox4x32_10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4]) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // both halves of each 32 x 32 -> 64-bit product from one multiply (v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * x0, p1 = (uint64_t)0xCD9E8D57u * x2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

// polynomial k of the moment basis at velocity (cx, cy, cz) (folded at compile time)
constexpr float mode_poly(int k, int cx, int cy, int cz) {
  const float x = (float)cx, y = (float)cy, z = (float)cz, c2 = x * x + y * y + z * z;
  return k == 4    ? c2 - 1.f
         : k == 5  ? 3.f * x * x - c2
         : k == 6  ? y * y - z * z
         : k == 7  ? x * y
         : k == 8  ? y * z
         : k == 9  ? z * x
         : k == 10 ? (3.f * c2 - 5.f) * x
         : k == 11 ? (3.f * c2 - 5.f) * y
         : k == 12 ? (3.f * c2 - 5.f) * z
         : k == 13 ? (y * y - z * z) * x
         : k == 14 ? (z * z - x * x) * y
         : k == 15 ? (x * x - y * y) * z
         : k == 16 ? 3.f * c2 * c2 - 6.f * c2 + 1.f
         : k == 17 ? (2.f * c2 - 3.f) * (3.f * x * x - c2)
                   : (2.f * c2 - 3.f) * (y * y - z * z);
}

constexpr float mode_inv_sqrt_norm(int k) {
  // 1 / sqrt(b_k), b_k = sum_i w_i e_k(c_i)^2 for k = 4 .. 18
  return k == 4 || k == 10 || k == 11 || k == 12 ? 1.2247448713915890f     // b = 2/3
         : k == 5 || k == 17                     ? 0.8660254037844386f     // b = 4/3
         : k == 6 || k == 18                     ? 1.5f                    // b = 4/9
         : k >= 7 && k <= 9                      ? 3.0f                    // b = 1/9
         : k >= 13 && k <= 15                    ? 2.1213203435596424f     // b = 2/9
                                                 : 0.7071067811865476f;    // b = 2 (k = 16)
}

// D3Q27 non-conserved modes k = 4..26 as codes a + 3 b + 9 c of their factor indices
// (P_a(c_x) P_b(c_y) P_c(c_z)), in increasing code
constexpr int MODE27_CODE[23] = {2, 4, 5, 6, 7, 8, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20,
                                 21, 22, 23, 24, 25, 26};

constexpr float poly3(int a, int c) { return a == 0 ? 1.f : (a == 1 ? (float)c : 3.f * c * c - 1.f); }
// 1 / sqrt of the factor norms 1, 1/3, 2
constexpr float inv_sqrt_norm3(int a) { return a == 0 ? 1.f : (a == 1 ? 1.7320508075688772f : 0.7071067811865476f); }

// D3Q27 mode k (4..26) at velocity (cx, cy, cz), divided by sqrt(b_k); folded at compile time
constexpr float mode27_scaled(int k, int cx, int cy, int cz) {
  const int code = MODE27_CODE[k - 4];
  const int a = code % 3, b = (code / 3) % 3, c = code / 9;
  return poly3(a, cx) * poly3(b, cy) * poly3(c, cz) * inv_sqrt_norm3(a) * inv_sqrt_norm3(b) *
         inv_sqrt_norm3(c);
}

// odd under c -> -c: an odd number of P_1 factors
constexpr bool mode27_odd(int k) {
  const int code = MODE27_CODE[k - 4];
  return (((code % 3) == 1) + (((code / 3) % 3) == 1) + ((code / 9) == 1)) % 2 == 1;
}

// the 4 NC normals of one site and step (NC = 4 for D3Q19, 6 for D3Q27)
template <int NC = 4>
__device__ __forceinline__ void site_normals(uint32_t seed0, uint32_t seed1, int64_t step, int site,
                                             float z[4 * NC]) {
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    uint32_t w[4];
    philox4x32_10((uint32_t)site, (uint32_t)((uint64_t)step & 0xffffffffu), (uint32_t)((uint64_t)step >> 32),
                  (uint32_t)q, seed0, seed1, w);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const float ua = ((float)(w[2 * t] >> 8) + 0.5f) * (1.0f / 16777216.0f);
      const float ub = ((float)(w[2 * t + 1] >> 8) + 0.5f) * (1.0f / 16777216.0f);
      // the hardware's transcendental units: v_log_f32 gives log2 (ua >= 2^-25 is a normal
      // number), v_sin_f32 / v_cos_f32 take the angle in turns, so 2 pi ub is ub itself
      // (each within about 2 ulp of the exact value)
      const float r = sqrtf(-2.0f * 0.693147180559945f * __builtin_amdgcn_logf(ua));
      const float sn = __builtin_amdgcn_sinf(ub), cs = __builtin_amdgcn_cosf(ub);
      z[4 * q + 2 * t] = r * cs;
      z[4 * q + 2 * t + 1] = r * sn;
    }
  }
}

// The unit-amplitude noise patterns of one site and step: pe from the modes even under
// c -> -c, po from the odd ones (D3Q19: k = 10..15); the noise is A+ pe + A- po, with
// A- = A+ unless the two-relaxation-time collision relaxes the odd modes at omega-.
template <int Q = 19>
__device__ __forceinline__ void noise_patterns(uint32_t seed0, uint32_t seed1, int64_t step, int site,
                                               float pe[Q], float po[Q]) {
  constexpr int NC = Q == 27 ? 6 : 4;
  float z[4 * NC];
  site_normals<NC>(seed0, seed1, step, site, z);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    float ae = 0.f, ao = 0.f;
#pragma unroll
    for (int k = 4; k < Q; ++k) {
      const float e = Q == 27 ? mode27_scaled(k, CX[i], CY[i], CZ[i])
                              : mode_poly(k, CX[i], CY[i], CZ[i]) * mode_inv_sqrt_norm(k);
      const bool odd = Q == 27 ? mode27_odd(k) : (k >= 10 && k <= 15);
      if (e != 0.f) {
        if (odd) ao += e * z[k - 4];
        else ae += e * z[k - 4];
      }
    }
    pe[i] = wq<Q>(i) * ae;
    po[i] = wq<Q>(i) * ao;
  }
}

// noise amplitude A(rho, omega)
__device__ __forceinline__ float noise_amp(float kT, float rho, float omega) {
  const float g = 1.0f - omega;
  return sqrtf(3.0f * rho * kT * (1.0f - g * g));
}

// opposite velocity index: c_opp(i) = -c_i
constexpr int OPP(int i) { return i == 0 ? 0 : (i % 2 ? i + 1 : i - 1); }

// The two-relaxation-time variant: with d_i = g_i - g_eq_i + s_i/2 (s_i the Guo source before
// its prefactor) split into parts even and odd under c -> -c,
//   g*_i = g_i + s_i - omega+ d+_i - omega- d-_i = g_i + s_i - a d_i - b d_opp(i),
// a = (omega+ + omega-)/2, b = (omega+ - omega-)/2; omega- = omega+ is the BGK collision.
template <int Q = 19>
__device__ __forceinline__ bool collide_trt(float g[Q], float Fx, float Fy, float Fz, float rho0,
                                            float omega_p, float omega_m) {
  float drho, jx, jy, jz;
  moments<Q>(g, drho, jx, jy, jz);
  const float rho = rho0 + drho;
  const float inv = 1.0f / rho;
  const float ux = (jx + 0.5f * Fx) * inv;
  const float uy = (jy + 0.5f * Fy) * inv;
  const float uz = (jz + 0.5f * Fz) * inv;
  const float uu = ux * ux + uy * uy + uz * uz;
  const float uF = ux * Fx + uy * Fy + uz * Fz;
  const float base = drho - 1.5f * rho * uu;
  float d[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float cu = cdot<0>(ux, uy, uz, CX[i], CY[i], CZ[i]);
    const float cF = cdot<0>(Fx, Fy, Fz, CX[i], CY[i], CZ[i]);
    const float geq = wq<Q>(i) * (base + rho * (3.0f * cu + 4.5f * cu * cu));
    const float si = wq<Q>(i) * (3.0f * (cF - uF) + 9.0f * cu * cF);
    d[i] = g[i] - geq + 0.5f * si;
    g[i] += si;
  }
  const float a = 0.5f * (omega_p + omega_m), b = 0.5f * (omega_p - omega_m);
#pragma unroll
  for (int i = 0; i < Q; ++i) g[i] -= a * d[i] + b * d[OPP(i)];
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
