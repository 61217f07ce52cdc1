// lbmd_oracle.cpp -- plain, slow CPU reference of the coupled lattice-Boltzmann / atom step.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this file:
// it exists so that tests, the smoke check and the benchmark's CPU baseline can compare
// the HIP path against an independent implementation written from the paper.  It shares
// no code, header or table with the HIP library.
//
// What it follows (Lauricella et al., arXiv 2305.05025, Section 2.2 "Coupled Lattice
// Boltzmann and Molecular Dynamics"):
//   * Eq. (1), the single-relaxation-time (BGK) lattice Boltzmann equation on the
//     19-speed D3Q19 lattice, with relaxation frequency omega = 2/(6 nu + 1), i.e.
//     tau = 1/omega = 3 nu + 1/2 in lattice units, and the second-order (in Mach number)
//     truncated Maxwell-Boltzmann equilibrium.  The printed sign of the relaxation term is
//     read as the standard BGK "minus omega (f - f_eq)" (the printed plus sign would make
//     the non-equilibrium part grow by (1 + omega) per step).
//   * Eqs. (2)-(3): rho = sum_i f_i, rho u = sum_i f_i c_i.
//   * The forcing term S_i of Eq. (1), here the Guo-Zheng-Shi scheme (Phys. Rev. E 65,
//     046308, 2002) because the paper leaves the scheme open.
//   * The thermal noise xi_i of the source term (fluctuating LB after Adhikari et al. 2005,
//     which the paper cites), off when kT = 0: Gaussian noise on the 15 non-conserved modes
//     of an orthogonal D3Q19 moment basis (Duenweg, Schiller & Ladd, Phys. Rev. E 76,
//     036704, 2007), each with variance mu b_k (1 - (1 - omega)^2), mu = rho kT / c_s^2,
//     rho the local density before the collision.  The normals come from the counter-based
//     generator Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11) keyed by the seed and
//     counted by (site, step), so that any implementation of the same definition draws the
//     same noise.
//   * The friction coupling paragraph: fluid velocity at an atom by linear interpolation
//     over the nearest eight lattice nodes, friction force gamma (u - v), the equal and
//     opposite force entering the lattice through S_i with the same (trilinear) weights,
//     one lattice step per atom step.
//
// The atom force field of the paper (CHARMM36 + implicit-solvent Coulomb) is replaced by
// a stand-in: harmonic tethers to the initial positions, harmonic chain bonds, a
// Lennard-Jones pair term cut off at r_c with minimum image and shifted so that its force
// vanishes continuously at r_c, bonded pairs optionally excluded, and the paper's
// implicit-solvent Coulomb term (direct summation with a distance-dependent permittivity, i.e.
// one more 1/r: U = k_C q_i q_j / r^2) under the same cut-off, shift and exclusions.  Atom update: symplectic Euler, v += F/m then x += v (dt = 1).
//
// Populations are kept as deviations g_i = f_i - w_i rho0 (exactly the same scheme,
// written around the rest state).  All arithmetic is in the template scalar T:
// double (the oracle proper), float (to measure the FP32 error floor) or Dual (forward-mode
// derivative of a loss with respect to gamma, tau or a body-force direction).
//
// Velocity sets: the paper's D3Q19, and (as the higher-order set its outlook in Section 4
// proposes) the 27-speed D3Q27 with the same equilibrium, forcing and collision written over
// its velocities and weights.  Its thermal noise uses the orthogonal tensor-product basis of
// the one-dimensional three-speed polynomials (1, c, 3 c^2 - 1) in place of the D3Q19 basis.
//
// Parity status: every sub-step is pinned by the CPU tests (closed forms, invariants,
// brute force); the long coupled trajectory itself has no published values to pin
// against beyond those invariants.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <array>

#include <omp.h>

namespace {

// ---------------------------------------------------------------------------------------
// Velocity sets.  D3Q19: the rest velocity, the 6 face neighbours and the 12 edge
// neighbours (the first 19 rows below).  D3Q27 adds the 8 corner neighbours.
// Ordering: opposite(i) = i + 1 for odd i, i - 1 for even i > 0.
// Weights: D3Q19 1/3, 1/18, 1/36; D3Q27 8/27, 2/27, 1/54, 1/216 (rest, face, edge, corner).
// ---------------------------------------------------------------------------------------
constexpr int QMAX = 27;
const int CV[QMAX][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};
const double WV19[19] = {
    1.0 / 3.0,
    1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
    1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
const double WV27[27] = {
    8.0 / 27.0,
    2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0,
    1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
    1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
    1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0,
    1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0};
// weight w_i of velocity set Q (19 or 27)
inline double wq(int Q, int i) { return Q == 27 ? WV27[i] : WV19[i]; }
// the D3Q19 weights (the moment basis of the thermal noise is defined on them)
inline double WV(int i) { return WV19[i]; }

// ---------------------------------------------------------------------------------------
// Forward-mode dual number: value + derivative along one seeded direction.
// ---------------------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual(double a = 0.0, double b = 0.0) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }

inline double val(double x) { return x; }
inline double val(float x) { return x; }
inline double val(const Dual& x) { return x.v; }
inline double dval(const Dual& x) { return x.d; }

inline double sqrtT(double x) { return std::sqrt(x); }
inline float sqrtT(float x) { return std::sqrt(x); }
inline Dual sqrtT(Dual x) { return sqrt(x); }

// ---------------------------------------------------------------------------------------
// Problem description (scalars in T so that gamma / tau can carry derivatives).
// ---------------------------------------------------------------------------------------
template <class T>
struct Model {
  int Q = 19;                                // velocity set: 19 or 27
  int L[3];
  long S;
  long P;                                    // plane stride of the population arrays held here
  T tau, rho0, gamma, mass, k_tether, k_bond, r0_bond, lj_eps, lj_sigma, lj_rc;
  T coul_k;                                  // implicit-solvent Coulomb prefactor (0: off)
  T trt_magic;                               // two-relaxation-time magic parameter (0: BGK)
  std::vector<T> charge;                     // per atom
  double kT;                                 // thermal energy (0: no noise)
  uint32_t seed[2];                          // Philox key
  int lj_exclude_bonded;
  int n_atoms, n_bonds;
  std::vector<int> bond_i, bond_j;           // bond list
  std::vector<std::vector<int>> partners;    // bonded partners per atom (for exclusions)
  std::vector<T> fext;                       // external force density [3][S]
  std::vector<T> anchor;                     // tether anchors = initial positions [N][3]
};

template <class T>
struct State {
  int64_t step = 0;   // step index (counts the noise)
  std::vector<T> g;   // pre-collision populations, deviation form, [Q][P] (sites 0..S-1 used)
  std::vector<T> X;   // unwrapped positions [N][3]
  std::vector<T> V;   // velocities [N][3]
};

inline long site_index(const int L[3], long x, long y, long z) { return x + L[0] * (y + (long)L[1] * z); }

// Population arrays held by the oracle keep their Q planes a few cache lines more than S
// apart: with a power-of-two S every site's Q values would otherwise share one cache set
// and the site loops run an order of magnitude slower.  Storage only; the values are those
// of the caller's [Q][S] arrays.
inline long plane_stride(long S) { return S + 8; }

template <class T>
void set_geometry(int Q, const int32_t* L, Model<T>& m) {
  m.Q = Q;
  for (int a = 0; a < 3; ++a) m.L[a] = L[a];
  m.S = (long)L[0] * L[1] * L[2];
  m.P = plane_stride(m.S);
}

// caller [Q][S] <-> oracle [Q][P]
template <class T>
void load_pops(const Model<T>& m, const double* g, std::vector<T>& out) {
  out.assign((size_t)m.Q * m.P, T(0.0));
  for (int i = 0; i < m.Q; ++i)
    for (long x = 0; x < m.S; ++x) out[i * m.P + x] = T(g[i * m.S + x]);
}
template <class T>
void store_pops(const Model<T>& m, const std::vector<T>& in, double* g) {
  for (int i = 0; i < m.Q; ++i)
    for (long x = 0; x < m.S; ++x) g[i * m.S + x] = val(in[i * m.P + x]);
}

inline long wrap(long a, int n) {
  long r = a % n;
  return r < 0 ? r + n : r;
}

// Eqs. (2)-(3) in deviation form: delta rho = sum_i g_i, j = sum_i c_i g_i.
template <class T>
void moments_at(const Model<T>& m, const std::vector<T>& g, long s, T& drho, T j[3]) {
  drho = T(0.0);
  j[0] = j[1] = j[2] = T(0.0);
  for (int i = 0; i < m.Q; ++i) {
    T gi = g[i * m.P + s];
    drho += gi;
    j[0] += T((double)CV[i][0]) * gi;
    j[1] += T((double)CV[i][1]) * gi;
    j[2] += T((double)CV[i][2]) * gi;
  }
}

// Second-order equilibrium (Section 2.2 after Eq. 1), minus its rest part w_i rho0:
//   g_eq_i = w_i [ delta_rho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u) ].
template <class T>
void equilibrium_dev(int Q, T drho, T rho, const T u[3], T out[]) {
  T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < Q; ++i) {
    T cu = T((double)CV[i][0]) * u[0] + T((double)CV[i][1]) * u[1] + T((double)CV[i][2]) * u[2];
    out[i] = T(wq(Q, i)) * (drho + rho * (T(3.0) * cu + T(4.5) * cu * cu - T(1.5) * uu));
  }
}

// Opposite velocity: c_opp(i) = -c_i.
inline int opposite(int i) { return i == 0 ? 0 : (i % 2 ? i + 1 : i - 1); }

// Relaxation rate of the antisymmetric part (two-relaxation-time collision) from the
// "magic" parameter Lambda = (1/omega+ - 1/2)(1/omega- - 1/2), omega+ = 1/tau.
template <class T>
T omega_minus(T tau, T magic) {
  return T(1.0) / (T(0.5) + magic / (tau - T(0.5)));
}

// Eq. (1) at one node with Guo forcing:
//   u* = (j + F/2) / rho
//   s_i = w_i [ 3 (c_i - u*) + 9 (c_i . u*) c_i ] . F
//   BGK (magic = 0): g*_i = g_i - (g_i - g_eq_i(rho, u*)) / tau + (1 - 1/(2 tau)) s_i
//   two relaxation times (magic > 0; the collision-variant extension): with
//     d_i = g_i - g_eq_i + s_i / 2 split into its parts even and odd under c -> -c,
//     g*_i = g_i + s_i - omega+ d+_i - omega- d-_i,  omega+ = 1/tau, omega- from magic,
//   which is the BGK form above when omega- = omega+.
template <class T>
void collide_node(int Q, T tau, T rho0, const T g[], const T F[3], T out[], T magic = T(0.0)) {
  T drho = T(0.0), j[3] = {T(0.0), T(0.0), T(0.0)};
  for (int i = 0; i < Q; ++i) {
    drho += g[i];
    for (int a = 0; a < 3; ++a) j[a] += T((double)CV[i][a]) * g[i];
  }
  T rho = rho0 + drho;
  T u[3];
  for (int a = 0; a < 3; ++a) u[a] = (j[a] + T(0.5) * F[a]) / rho;
  T geq[QMAX];
  equilibrium_dev(Q, drho, rho, u, geq);
  T pref = T(1.0) - T(1.0) / (T(2.0) * tau);
  T sraw[QMAX];
  for (int i = 0; i < Q; ++i) {
    T cu = T((double)CV[i][0]) * u[0] + T((double)CV[i][1]) * u[1] + T((double)CV[i][2]) * u[2];
    T src = T(0.0);
    for (int a = 0; a < 3; ++a) {
      T ca = T((double)CV[i][a]);
      src += (T(3.0) * (ca - u[a]) + T(9.0) * cu * ca) * F[a];
    }
    T Si = pref * T(wq(Q, i)) * src;
    out[i] = g[i] - (g[i] - geq[i]) / tau + Si;
    sraw[i] = T(wq(Q, i)) * src;
  }
  if (val(magic) > 0.0) {
    const T om_p = T(1.0) / tau, om_m = omega_minus(tau, magic);
    T d[QMAX];
    for (int i = 0; i < Q; ++i) d[i] = g[i] - geq[i] + T(0.5) * sraw[i];
    for (int i = 0; i < Q; ++i) {
      const T dp = T(0.5) * (d[i] + d[opposite(i)]);
      const T dm = T(0.5) * (d[i] - d[opposite(i)]);
      out[i] = g[i] + sraw[i] - om_p * dp - om_m * dm;
    }
  }
}

// Left-hand side of Eq. (1): the value leaving node x along c_i arrives at x + c_i
// (periodic box).
template <class T>
void stream(const Model<T>& m, const std::vector<T>& post, std::vector<T>& pre) {
  const int* L = m.L;
  for (int i = 0; i < m.Q; ++i)
#pragma omp parallel for schedule(static)
    for (long z = 0; z < L[2]; ++z)
      for (long y = 0; y < L[1]; ++y)
        for (long x = 0; x < L[0]; ++x) {
          long src = site_index(L, x, y, z);
          long dst = site_index(L, wrap(x + CV[i][0], L[0]), wrap(y + CV[i][1], L[1]),
                                wrap(z + CV[i][2], L[2]));
          pre[i * m.P + dst] = post[i * m.P + src];
        }
}

// The eight lattice nodes around a point and their trilinear weights.  The point is
// first brought into the box [0, L) by floor-mod; nodes sit at integer coordinates.
template <class T>
void stencil(const int L[3], const T* Xa, long node[8], T w[8]) {
  long i0[3];
  T d[3];
  for (int a = 0; a < 3; ++a) {
    T Y = Xa[a] - T((double)L[a]) * T(std::floor(val(Xa[a]) / L[a]));
    double fl = std::floor(val(Y));
    d[a] = Y - T(fl);
    i0[a] = wrap((long)fl, L[a]);
  }
  for (int k = 0; k < 8; ++k) {
    int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
    T wx = dx ? d[0] : T(1.0) - d[0];
    T wy = dy ? d[1] : T(1.0) - d[1];
    T wz = dz ? d[2] : T(1.0) - d[2];
    w[k] = wx * wy * wz;
    node[k] = site_index(L, wrap(i0[0] + dx, L[0]), wrap(i0[1] + dy, L[1]), wrap(i0[2] + dz, L[2]));
  }
}

// Linear interpolation over the nearest eight nodes of a [3][S] field at atom positions.
template <class T>
void interpolate(const int L[3], long S, const std::vector<T>& field, int n, const T* X, T* U) {
  for (int a = 0; a < n; ++a) {
    long node[8];
    T w[8];
    stencil(L, &X[3 * a], node, w);
    for (int c = 0; c < 3; ++c) {
      T acc = T(0.0);
      for (int k = 0; k < 8; ++k) acc += w[k] * field[c * S + node[k]];
      U[3 * a + c] = acc;
    }
  }
}

// Transpose of the interpolation: field(node) += W(X_a, node) F_a.
template <class T>
void spread(const int L[3], long S, int n, const T* X, const T* F, std::vector<T>& field) {
  for (int a = 0; a < n; ++a) {
    long node[8];
    T w[8];
    stencil(L, &X[3 * a], node, w);
    for (int k = 0; k < 8; ++k)
      for (int c = 0; c < 3; ++c) field[c * S + node[k]] += w[k] * F[3 * a + c];
  }
}

// ---------------------------------------------------------------------------------------
// Thermal noise.
// Philox4x32-10: ten rounds of (L0, R0, L1, R1) -> (hi(M1 R1) ^ L1 ^ k0, lo(M1 R1),
// hi(M0 R0) ^ L0' ^ k1, lo(M0 R0)) on the counter (x0, x1, x2, x3), with the key bumped by
// the Weyl constants between rounds.
// ---------------------------------------------------------------------------------------
void philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * x[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * x[2];
    const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x[1] ^ k0;
    const uint32_t y1 = (uint32_t)p1;
    const uint32_t y2 = (uint32_t)(p0 >> 32) ^ x[3] ^ k1;
    const uint32_t y3 = (uint32_t)p0;
    x[0] = y0;
    x[1] = y1;
    x[2] = y2;
    x[3] = y3;
  }
  for (int q = 0; q < 4; ++q) out[q] = x[q];
}

// 4 ncalls standard normals for one site and step (ncalls = 4 for D3Q19, 6 for D3Q27):
// Philox counters (site, step low word, step high word, q) for q = 0..ncalls-1 under the
// seed; each output word w gives the uniform u = (floor(w / 2^8) + 1/2) / 2^24 in (0, 1),
// and consecutive pairs (u_a, u_b) give sqrt(-2 ln u_a) (cos 2 pi u_b, sin 2 pi u_b)
// (Box-Muller).
void site_normals(const uint32_t seed[2], int64_t step, long site, double z[], int ncalls = 4) {
  for (int q = 0; q < ncalls; ++q) {
    const uint32_t ctr[4] = {(uint32_t)site, (uint32_t)((uint64_t)step & 0xffffffffu),
                             (uint32_t)((uint64_t)step >> 32), (uint32_t)q};
    uint32_t w[4];
    philox4x32_10(ctr, seed, w);
    double u[4];
    for (int t = 0; t < 4; ++t) u[t] = ((double)(w[t] >> 8) + 0.5) / 16777216.0;
    for (int t = 0; t < 2; ++t) {
      const double r = std::sqrt(-2.0 * std::log(u[2 * t]));
      const double th = 2.0 * M_PI * u[2 * t + 1];
      z[4 * q + 2 * t] = r * std::cos(th);
      z[4 * q + 2 * t + 1] = r * std::sin(th);
    }
  }
}

// The moment basis: e_k(c) for k = 0..18, polynomials of the velocity c: density, momentum,
// bulk and shear stresses, then nine kinetic ("ghost") modes.  Orthogonal under the weights:
// sum_i w_i e_k(c_i) e_l(c_i) = b_k delta_kl.
double mode_poly(int k, const int c[3]) {
  const double x = c[0], y = c[1], z = c[2], c2 = x * x + y * y + z * z;
  switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return c2 - 1.0;
    case 5: return 3.0 * x * x - c2;
    case 6: return y * y - z * z;
    case 7: return x * y;
    case 8: return y * z;
    case 9: return z * x;
    case 10: return (3.0 * c2 - 5.0) * x;
    case 11: return (3.0 * c2 - 5.0) * y;
    case 12: return (3.0 * c2 - 5.0) * z;
    case 13: return (y * y - z * z) * x;
    case 14: return (z * z - x * x) * y;
    case 15: return (x * x - y * y) * z;
    case 16: return 3.0 * c2 * c2 - 6.0 * c2 + 1.0;
    case 17: return (2.0 * c2 - 3.0) * (3.0 * x * x - c2);
    default: return (2.0 * c2 - 3.0) * (y * y - z * z);
  }
}

// (the tables below are built once, on first use, by thread-safe static initialisation)
double mode_norm(int k) {
  static const std::array<double, 19> b = [] {
    std::array<double, 19> t{};
    for (int q = 0; q < 19; ++q) {
      double acc = 0.0;
      for (int i = 0; i < 19; ++i) acc += WV(i) * mode_poly(q, CV[i]) * mode_poly(q, CV[i]);
      t[q] = acc;
    }
    return t;
  }();
  return b[k];
}

// The D3Q27 moment basis: products of the one-dimensional polynomials P_0 = 1, P_1 = c,
// P_2 = 3 c^2 - 1, orthogonal under the three-speed weights (2/3, 1/6, 1/6) with norms
// 1, 1/3, 2; so e_(a,b,c)(c) = P_a(c_x) P_b(c_y) P_c(c_z) is orthogonal under the D3Q27
// weights with norm n_a n_b n_c.  Ordering: k = 0 density (0,0,0); 1..3 momentum (1,0,0),
// (0,1,0), (0,0,1); then the other 23 triples by increasing a + 3 b + 9 c.  A mode is odd
// under c -> -c when an odd number of its factors are P_1.
void mode27_triple(int k, int abc[3]) {
  static const std::array<std::array<int, 3>, 27> tab = [] {
    std::array<std::array<int, 3>, 27> t{};
    const int first[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int q = 0; q < 4; ++q)
      for (int d = 0; d < 3; ++d) t[q][d] = first[q][d];
    int n = 4;
    for (int code = 0; code < 27; ++code) {
      const int a = code % 3, b = (code / 3) % 3, c = code / 9;
      if (a + b + c <= 1) continue;   // the four conserved modes above
      t[n][0] = a;
      t[n][1] = b;
      t[n][2] = c;
      ++n;
    }
    return t;
  }();
  for (int d = 0; d < 3; ++d) abc[d] = tab[k][d];
}

double poly1d(int a, int c) { return a == 0 ? 1.0 : (a == 1 ? (double)c : 3.0 * c * c - 1.0); }

double mode27_poly(int k, const int c[3]) {
  int abc[3];
  mode27_triple(k, abc);
  return poly1d(abc[0], c[0]) * poly1d(abc[1], c[1]) * poly1d(abc[2], c[2]);
}

bool mode27_odd(int k) {
  int abc[3];
  mode27_triple(k, abc);
  return ((abc[0] == 1) + (abc[1] == 1) + (abc[2] == 1)) % 2 == 1;
}

double mode27_norm(int k) {
  static const std::array<double, 27> b = [] {
    std::array<double, 27> t{};
    for (int q = 0; q < 27; ++q) {
      double acc = 0.0;
      for (int i = 0; i < 27; ++i) acc += WV27[i] * mode27_poly(q, CV[i]) * mode27_poly(q, CV[i]);
      t[q] = acc;
    }
    return t;
  }();
  return b[k];
}

// Noise added to the post-collision populations at one site (Q = 19 or 27 velocities):
//   xi_i = w_i sum_{k=4..Q-1} e_k(c_i) phi_k z_{k-4} / b_k,
//   phi_k = sqrt(mu b_k (1 - (1 - omega_k)^2)),  mu = 3 rho kT,
// omega_k the rate that relaxes mode k: 1/tau, except the modes odd under c -> -c (D3Q19:
// k = 10..15) under the two-relaxation-time collision, which relax at omega-.
template <class T>
void site_noise(int Q, double kT, T tau, T rho, const uint32_t seed[2], int64_t step, long site,
                T xi[], T magic = T(0.0)) {
  double z[24];
  site_normals(seed, step, site, z, Q == 27 ? 6 : 4);
  const T om_p = T(1.0) / tau;
  const T om_m = val(magic) > 0.0 ? omega_minus(tau, magic) : om_p;
  const T gp = T(1.0) - om_p, gm = T(1.0) - om_m;
  const T amp2_p = T(3.0 * kT) * rho * (T(1.0) - gp * gp);
  const T amp2_m = T(3.0 * kT) * rho * (T(1.0) - gm * gm);
  for (int i = 0; i < Q; ++i) {
    T acc = T(0.0);
    for (int k = 4; k < Q; ++k) {
      const double b = Q == 27 ? mode27_norm(k) : mode_norm(k);
      const bool odd = Q == 27 ? mode27_odd(k) : (k >= 10 && k <= 15);
      const double e = Q == 27 ? mode27_poly(k, CV[i]) : mode_poly(k, CV[i]);
      const T amp2 = odd ? amp2_m : amp2_p;
      acc += T(e * z[k - 4]) * sqrtT(amp2 * T(b)) / T(b);
    }
    xi[i] = T(wq(Q, i)) * acc;
  }
}

template <class T>
T min_image(T r, int L) {
  return r - T((double)L) * T(std::floor(val(r) / L + 0.5));
}

template <class T>
bool bonded(const Model<T>& m, int i, int j) {
  for (int p : m.partners[i])
    if (p == j) return true;
  return false;
}

template <class T>
bool pair_terms_on(const Model<T>& m) {
  return val(m.lj_eps) != 0.0 || val(m.coul_k) != 0.0;
}

// The pair terms act below the cut-off r_c and are shifted so that the force falls to zero
// continuously there (the paper gives its runs a cut-off distance only, Section 2.2; an
// unshifted truncation makes the force jump at r_c, and then whether a pair within rounding of
// r_c counts decides a finite force difference).  With the unshifted terms written as
// F_i = g0(r^2) r (r = X_i - X_j):
//   LJ: U0 = 4 eps [(s/r)^12 - (s/r)^6],  g0 = 24 eps / r^2 [2 (s/r)^12 - (s/r)^6];
//   implicit-solvent Coulomb (permittivity ~ r): U0 = k_C q_i q_j / r^2,  g0 = 2 k_C q_i q_j / r^4;
// each term below r_c is
//   g(r^2) = g0(r^2) - g0(r_c^2),   U(r^2) = U0(r^2) - U0(r_c^2) + g0(r_c^2) (r^2 - r_c^2) / 2,
// so that F = -grad U, and F and U are continuous and zero at r_c.
template <class T>
T lj_g0(const Model<T>& m, T r2) {
  T sr2 = m.lj_sigma * m.lj_sigma / r2;
  T sr6 = sr2 * sr2 * sr2;
  return T(24.0) * m.lj_eps * (T(2.0) * sr6 * sr6 - sr6) / r2;
}

template <class T>
T lj_u0(const Model<T>& m, T r2) {
  T sr6 = (m.lj_sigma * m.lj_sigma / r2) * (m.lj_sigma * m.lj_sigma / r2) * (m.lj_sigma * m.lj_sigma / r2);
  return T(4.0) * m.lj_eps * (sr6 * sr6 - sr6);
}

// |F_i| / |r| of the pair terms at squared distance r2 < r_c^2 (force on i along r)
template <class T>
T pair_force_over_r(const Model<T>& m, int i, int j, T r2) {
  const T rc2 = m.lj_rc * m.lj_rc;
  T f = T(0.0);
  if (val(m.lj_eps) != 0.0) f += lj_g0(m, r2) - lj_g0(m, rc2);
  if (val(m.coul_k) != 0.0) {
    const T kqq2 = T(2.0) * m.coul_k * m.charge[i] * m.charge[j];
    f += kqq2 / (r2 * r2) - kqq2 / (rc2 * rc2);
  }
  return f;
}

template <class T>
T pair_energy(const Model<T>& m, int i, int j, T r2) {
  const T rc2 = m.lj_rc * m.lj_rc;
  T e = T(0.0);
  if (val(m.lj_eps) != 0.0) e += lj_u0(m, r2) - lj_u0(m, rc2) + T(0.5) * lj_g0(m, rc2) * (r2 - rc2);
  if (val(m.coul_k) != 0.0) {
    const T kqq = m.coul_k * m.charge[i] * m.charge[j];
    e += kqq / r2 - kqq / rc2 + kqq / (rc2 * rc2) * (r2 - rc2);
  }
  return e;
}

// Stand-in force field at positions X (unwrapped): tethers, bonds, cut-off pair terms.
template <class T>
void atom_forces(const Model<T>& m, const std::vector<T>& X, std::vector<T>& F) {
  const int N = m.n_atoms;
  std::fill(F.begin(), F.end(), T(0.0));
  // harmonic tethers: U = k/2 |X - X^0|^2
  if (val(m.k_tether) != 0.0)
    for (int a = 0; a < N; ++a)
      for (int c = 0; c < 3; ++c) F[3 * a + c] -= m.k_tether * (X[3 * a + c] - m.anchor[3 * a + c]);
  // harmonic bonds: U = k/2 (r - r0)^2
  for (int b = 0; b < m.n_bonds; ++b) {
    int i = m.bond_i[b], j = m.bond_j[b];
    T r[3];
    for (int c = 0; c < 3; ++c) r[c] = min_image(X[3 * i + c] - X[3 * j + c], m.L[c]);
    T rl = sqrtT(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    T fmag = -m.k_bond * (rl - m.r0_bond) / rl;   // force on i along r = X_i - X_j
    for (int c = 0; c < 3; ++c) {
      F[3 * i + c] += fmag * r[c];
      F[3 * j + c] -= fmag * r[c];
    }
  }
  // Pair terms for r < r_c, all pairs (brute force): Lennard-Jones
  // U = 4 eps [(s/r)^12 - (s/r)^6] and implicit-solvent Coulomb U = k_C q_i q_j / r^2
  if (pair_terms_on(m)) {
    T rc2 = m.lj_rc * m.lj_rc;
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j) {
        T r[3];
        for (int c = 0; c < 3; ++c) r[c] = min_image(X[3 * i + c] - X[3 * j + c], m.L[c]);
        T r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (!(val(r2) < val(rc2))) continue;
        if (m.lj_exclude_bonded && bonded(m, i, j)) continue;
        T fmag = pair_force_over_r(m, i, j, r2);
        for (int c = 0; c < 3; ++c) {
          F[3 * i + c] += fmag * r[c];
          F[3 * j + c] -= fmag * r[c];
        }
      }
  }
}

// The same force field evaluated for one atom i only.  The pair partners are scanned in
// ascending index: all atoms, or (cand != NULL) the candidate list of i from pair_candidates,
// which holds every atom closer than r_c in ascending order, so the sum has the same terms in
// the same order.  Each partner's contribution is added to atom i's force in the order that
// the pairwise loop of atom_forces adds it (tether, bonds in list order, pairs by ascending
// partner), with the pair vector negated exactly, so the two give the same bits.
template <class T>
void atom_force_one(const Model<T>& m, const std::vector<T>& X, int i, T F[3],
                    const std::vector<int>* cand = nullptr) {
  F[0] = F[1] = F[2] = T(0.0);
  for (int c = 0; c < 3; ++c) F[c] -= m.k_tether * (X[3 * i + c] - m.anchor[3 * i + c]);
  for (int b = 0; b < m.n_bonds; ++b) {
    int p = m.bond_i[b], q = m.bond_j[b];
    if (p != i && q != i) continue;
    int j = p == i ? q : p;
    T r[3];
    for (int c = 0; c < 3; ++c) r[c] = min_image(X[3 * i + c] - X[3 * j + c], m.L[c]);
    T rl = sqrtT(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    T fmag = -m.k_bond * (rl - m.r0_bond) / rl;
    for (int c = 0; c < 3; ++c) F[c] += fmag * r[c];
  }
  if (pair_terms_on(m))
    for (int k = 0, n = cand ? (int)cand->size() : m.n_atoms; k < n; ++k) {
      const int j = cand ? (*cand)[k] : k;
      if (j == i) continue;
      T r[3];
      for (int c = 0; c < 3; ++c) r[c] = min_image(X[3 * i + c] - X[3 * j + c], m.L[c]);
      T r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
      if (!(val(r2) < val(m.lj_rc * m.lj_rc))) continue;
      if (m.lj_exclude_bonded && bonded(m, i, j)) continue;
      T fmag = pair_force_over_r(m, i, j, r2);
      for (int c = 0; c < 3; ++c) F[c] += fmag * r[c];
    }
}

// Pair candidates.  The pair terms act only below the cut-off r_c (minimum image).  Put the
// atoms into a periodic grid of cells at least 1.001 r_c wide (3 or more along every axis):
// any two atoms closer than r_c then sit in the same or in neighbouring cells (the margin
// exceeds the rounding of the cell index), so the atoms of the 3 x 3 x 3 cells around an
// atom's own, in ascending index, hold all of its partners in the order a scan of every atom
// meets them.  Returns false (scan every atom) when an axis has fewer than 3 cells, where
// neighbouring cells would repeat.
struct CellGrid {
  int nc[3] = {0, 0, 0};
  std::vector<std::vector<int>> atoms;   // per cell, ascending atom index
  std::vector<int> cell_of;              // per atom
};

template <class T>
bool build_cells(const Model<T>& m, const std::vector<T>& X, CellGrid& g) {
  const double rc = val(m.lj_rc);
  for (int a = 0; a < 3; ++a) {
    g.nc[a] = (int)std::floor((double)m.L[a] / (rc * 1.001));
    if (g.nc[a] < 3) return false;
  }
  g.atoms.assign((size_t)g.nc[0] * g.nc[1] * g.nc[2], {});
  g.cell_of.resize(m.n_atoms);
  for (int i = 0; i < m.n_atoms; ++i) {
    int q[3];
    for (int a = 0; a < 3; ++a) {
      const double x = val(X[3 * i + a]);
      const double y = x - m.L[a] * std::floor(x / m.L[a]);   // into [0, L)
      const int k = (int)std::floor(y * g.nc[a] / m.L[a]);
      q[a] = k < 0 ? 0 : (k >= g.nc[a] ? g.nc[a] - 1 : k);
    }
    const int c = q[0] + g.nc[0] * (q[1] + g.nc[1] * q[2]);
    g.atoms[c].push_back(i);   // i ascends, so each cell's list is sorted
    g.cell_of[i] = c;
  }
  return true;
}

// the atoms of the 27 cells around atom i's cell, ascending
inline void pair_candidates(const CellGrid& g, int i, std::vector<int>& out) {
  out.clear();
  const int c = g.cell_of[i];
  const int q[3] = {c % g.nc[0], (c / g.nc[0]) % g.nc[1], c / (g.nc[0] * g.nc[1])};
  for (int dz = -1; dz <= 1; ++dz)
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int x = (q[0] + dx + g.nc[0]) % g.nc[0], y = (q[1] + dy + g.nc[1]) % g.nc[1],
                  z = (q[2] + dz + g.nc[2]) % g.nc[2];
        const std::vector<int>& v = g.atoms[x + g.nc[0] * (y + g.nc[1] * z)];
        out.insert(out.end(), v.begin(), v.end());
      }
  std::sort(out.begin(), out.end());
}

// The force field at X evaluated atom by atom (atom_force_one, in parallel over atoms): the
// same values, bit for bit, as the pairwise loop of atom_forces.
template <class T>
void atom_forces_by_atom(const Model<T>& m, const std::vector<T>& X, std::vector<T>& F) {
  CellGrid g;
  const bool cells = pair_terms_on(m) && build_cells(m, X, g);
#pragma omp parallel
  {
    std::vector<int> cand;
#pragma omp for schedule(dynamic, 64)
    for (int i = 0; i < m.n_atoms; ++i) {
      if (cells) pair_candidates(g, i, cand);
      T f[3];
      atom_force_one(m, X, i, f, cells ? &cand : nullptr);
      for (int c = 0; c < 3; ++c) F[3 * i + c] = f[c];
    }
  }
}

template <class T>
T atom_energy(const Model<T>& m, const std::vector<T>& X) {
  const int N = m.n_atoms;
  T E = T(0.0);
  for (int a = 0; a < N; ++a)
    for (int c = 0; c < 3; ++c) {
      T d = X[3 * a + c] - m.anchor[3 * a + c];
      E += T(0.5) * m.k_tether * d * d;
    }
  for (int b = 0; b < m.n_bonds; ++b) {
    int i = m.bond_i[b], j = m.bond_j[b];
    T r[3];
    for (int c = 0; c < 3; ++c) r[c] = min_image(X[3 * i + c] - X[3 * j + c], m.L[c]);
    T rl = sqrtT(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    E += T(0.5) * m.k_bond * (rl - m.r0_bond) * (rl - m.r0_bond);
  }
  if (pair_terms_on(m))
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j) {
        T r[3];
        for (int c = 0; c < 3; ++c) r[c] = min_image(X[3 * i + c] - X[3 * j + c], m.L[c]);
        T r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (!(val(r2) < val(m.lj_rc * m.lj_rc))) continue;
        if (m.lj_exclude_bonded && bonded(m, i, j)) continue;
        E += pair_energy(m, i, j, r2);
      }
  return E;
}

// One coupled step, in this order:
//  1 moments at every node (pre-collision state of step n)
//  2 coupling velocity u_c = (j + F_ext/2) / rho (the atoms' own force is not included)
//  3 U_a = interpolation of u_c at X_a^n
//  4 friction on the atom F_c = gamma (U_a - v_a^n)
//  5 the fluid receives -F_c with the same trilinear weights: F = F_ext - spread(F_c)
//  6 BGK + Guo collision at every node with that F
//  7 streaming
//  8 stand-in force field at X^n
//  9 symplectic Euler: v^{n+1} = v^n + (F_ff + F_c)/m, X^{n+1} = X^n + v^{n+1}
// Arrays of a step, kept from step to step (allocating lattice-sized arrays anew every step
// costs more than the step's arithmetic on some hosts).
template <class T>
struct Work {
  std::vector<T> post;      // post-collision populations [Q][P]
  std::vector<T> uc;        // coupling velocity [3][S]
  std::vector<T> Fspread;   // spread friction force [3][S]
  std::vector<T> Ftot;      // total force density [3][S]
  std::vector<T> U, Fc, Fff;  // per atom [N][3]: interpolated velocity, friction, force field
  void size(const Model<T>& m) {
    post.resize((size_t)m.Q * m.P);
    uc.resize(3 * (size_t)m.S);
    Fspread.resize(3 * (size_t)m.S);
    Ftot.resize(3 * (size_t)m.S);
    U.resize(3 * (size_t)m.n_atoms);
    Fc.resize(3 * (size_t)m.n_atoms);
    Fff.resize(3 * (size_t)m.n_atoms);
  }
};

// Steps 1-5: friction force on every atom (w.Fc) and total force density on every node
// (w.Ftot).
template <class T>
void coupling_forces(const Model<T>& m, const State<T>& s, Work<T>& w) {
  const long S = m.S;
  const int N = m.n_atoms;
  std::vector<T>& uc = w.uc;
#pragma omp parallel for schedule(static)
  for (long x = 0; x < S; ++x) {
    T dr, j[3];
    moments_at(m, s.g, x, dr, j);
    T rho = m.rho0 + dr;
    for (int c = 0; c < 3; ++c) uc[c * S + x] = (j[c] + T(0.5) * m.fext[c * S + x]) / rho;
  }
  interpolate(m.L, S, uc, N, s.X.data(), w.U.data());
  for (int k = 0; k < 3 * N; ++k) w.Fc[k] = m.gamma * (w.U[k] - s.V[k]);
  std::fill(w.Fspread.begin(), w.Fspread.end(), T(0.0));
  spread(m.L, S, N, s.X.data(), w.Fc.data(), w.Fspread);
#pragma omp parallel for schedule(static)
  for (long k = 0; k < 3 * S; ++k) w.Ftot[k] = m.fext[k] - w.Fspread[k];
}

template <class T>
void coupled_step(const Model<T>& m, State<T>& s, Work<T>& w) {
  const long S = m.S;
  const int N = m.n_atoms;
  coupling_forces(m, s, w);
  std::vector<T>& Ftot = w.Ftot;
  std::vector<T>& scratch_post = w.post;
#pragma omp parallel for schedule(static)
  for (long x = 0; x < S; ++x) {
    T gin[QMAX], gout[QMAX], F[3];
    for (int i = 0; i < m.Q; ++i) gin[i] = s.g[i * m.P + x];
    for (int c = 0; c < 3; ++c) F[c] = Ftot[c * S + x];
    collide_node(m.Q, m.tau, m.rho0, gin, F, gout, m.trt_magic);
    if (m.kT > 0.0) {
      T rho = m.rho0;
      for (int i = 0; i < m.Q; ++i) rho += gin[i];
      T xi[QMAX];
      site_noise(m.Q, m.kT, m.tau, rho, m.seed, s.step, x, xi, m.trt_magic);
      for (int i = 0; i < m.Q; ++i) gout[i] += xi[i];
    }
    for (int i = 0; i < m.Q; ++i) scratch_post[i * m.P + x] = gout[i];
  }
  stream(m, scratch_post, s.g);
  atom_forces_by_atom(m, s.X, w.Fff);
  for (int k = 0; k < 3 * N; ++k) {
    s.V[k] = s.V[k] + (w.Fff[k] + w.Fc[k]) / m.mass;
    s.X[k] = s.X[k] + s.V[k];
  }
  s.step++;
}

}  // namespace

// =======================================================================================
// C interface (ctypes).  Arrays are float64 unless stated; layouts:
//   populations [Q][nz][ny][nx] (x fastest, Q = 19 or 27), fields [3][nz][ny][nx],
//   atoms [N][3].
// =======================================================================================
extern "C" {

struct or_params {
  int32_t L[3];
  int32_t n_atoms;
  int32_t n_bonds;
  int32_t lj_exclude_bonded;
  int32_t bf_kind;   // 0 none, 1 Kolmogorov sin(2 pi y / ny), 2 sign(y + 1/2 - ny/2), 3 field
  int32_t pad;
  double tau, rho0, gamma, mass, k_tether, k_bond, r0_bond, lj_eps, lj_sigma, lj_rc, bf_amp;
  double kT;          // thermal energy of the noise (0: none)
  uint32_t seed[2];   // Philox key
  int64_t step0;      // step index of the input state (counts the noise)
  double coul_k;      // implicit-solvent Coulomb prefactor k_C (0: off)
  const double* charge;   // [n_atoms] charges, or NULL (all zero)
  double trt_magic;   // two-relaxation-time collision: Lambda (0: BGK)
  int32_t velocity_set;   // 19 or 27 (0 means 19)
  int32_t pad2;
};

}  // extern "C"

namespace {

// the velocity set is 19 or 27 (or 0 for 19)
bool params_ok(const or_params* p) {
  const int q = p->velocity_set == 0 ? 19 : p->velocity_set;
  return q == 19 || q == 27;
}

inline int q_of(const or_params* p) { return p->velocity_set == 27 ? 27 : 19; }

template <class T>
void external_force(const or_params* p, const double* field, std::vector<T>& fext, long S) {
  fext.assign(3 * S, T(0.0));
  for (long z = 0; z < p->L[2]; ++z)
    for (long y = 0; y < p->L[1]; ++y)
      for (long x = 0; x < p->L[0]; ++x) {
        long s = site_index(p->L, x, y, z);
        double gx = 0.0;
        if (p->bf_kind == 1) {
          gx = p->bf_amp * std::sin(2.0 * M_PI * (double)y / (double)p->L[1]);
        } else if (p->bf_kind == 2) {
          double a = (double)y + 0.5 - 0.5 * (double)p->L[1];
          gx = p->bf_amp * (a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0));
        }
        if (p->bf_kind == 3) {
          for (int c = 0; c < 3; ++c) fext[c * S + s] = T(field[c * S + s]);
        } else {
          fext[0 * S + s] = T(gx);
        }
      }
}

template <class T>
void build_model(const or_params* p, const double* X0, const int32_t* bonds, const double* field,
                 Model<T>& m) {
  set_geometry(p->velocity_set == 27 ? 27 : 19, p->L, m);
  m.tau = T(p->tau);
  m.rho0 = T(p->rho0);
  m.gamma = T(p->gamma);
  m.mass = T(p->mass);
  m.k_tether = T(p->k_tether);
  m.k_bond = T(p->k_bond);
  m.r0_bond = T(p->r0_bond);
  m.lj_eps = T(p->lj_eps);
  m.lj_sigma = T(p->lj_sigma);
  m.lj_rc = T(p->lj_rc);
  m.lj_exclude_bonded = p->lj_exclude_bonded;
  m.kT = p->kT;
  m.coul_k = T(p->coul_k);
  m.trt_magic = T(p->trt_magic);
  m.charge.assign((size_t)p->n_atoms, T(0.0));
  if (p->charge)
    for (int a = 0; a < p->n_atoms; ++a) m.charge[a] = T(p->charge[a]);
  m.seed[0] = p->seed[0];
  m.seed[1] = p->seed[1];
  m.n_atoms = p->n_atoms;
  m.n_bonds = p->n_bonds;
  m.bond_i.resize(p->n_bonds);
  m.bond_j.resize(p->n_bonds);
  m.partners.assign(p->n_atoms, {});
  for (int b = 0; b < p->n_bonds; ++b) {
    m.bond_i[b] = bonds[2 * b];
    m.bond_j[b] = bonds[2 * b + 1];
    m.partners[bonds[2 * b]].push_back(bonds[2 * b + 1]);
    m.partners[bonds[2 * b + 1]].push_back(bonds[2 * b]);
  }
  m.anchor.resize(3 * (size_t)p->n_atoms);
  for (long k = 0; k < 3L * p->n_atoms; ++k) m.anchor[k] = T(X0[k]);
  external_force<T>(p, field, m.fext, m.S);
}

template <class T>
int run_impl(const or_params* p, double* g, double* X, double* V, const double* X0,
             const int32_t* bonds, const double* field, int32_t n_steps) {
  if (!params_ok(p)) return 2;
  Model<T> m;
  build_model<T>(p, X0, bonds, field, m);
  State<T> s;
  s.step = p->step0;
  load_pops(m, g, s.g);
  s.X.resize(3 * (size_t)m.n_atoms);
  s.V.resize(3 * (size_t)m.n_atoms);
  for (long k = 0; k < 3L * m.n_atoms; ++k) {
    s.X[k] = T(X[k]);
    s.V[k] = T(V[k]);
  }
  Work<T> w;
  w.size(m);
  for (int n = 0; n < n_steps; ++n) coupled_step(m, s, w);
  store_pops(m, s.g, g);
  for (long k = 0; k < 3L * m.n_atoms; ++k) {
    X[k] = val(s.X[k]);
    V[k] = val(s.V[k]);
  }
  return 0;
}

}  // namespace

extern "C" {

// threads the parallel loops of the oracle use (OpenMP's default team size)
int32_t or_num_threads() { return (int32_t)omp_get_max_threads(); }

void or_philox4x32_10(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
  philox4x32_10(ctr, key, out);
}

void or_site_normals(const uint32_t* seed, int64_t step, int64_t site, double* z) {
  site_normals(seed, step, (long)site, z);
}

// e[k * 19 + i] = e_k(c_i), b[k] = sum_i w_i e_k(c_i)^2
void or_mode_basis(double* e, double* b) {
  for (int k = 0; k < 19; ++k) {
    for (int i = 0; i < 19; ++i) e[k * 19 + i] = mode_poly(k, CV[i]);
    b[k] = mode_norm(k);
  }
}

void or_site_noise(double kT, double tau, double rho, const uint32_t* seed, int64_t step, int64_t site,
                   double* xi, double magic) {
  site_noise(19, kT, tau, rho, seed, step, (long)site, xi, magic);
}

void or_site_noise_q(int32_t q, double kT, double tau, double rho, const uint32_t* seed, int64_t step,
                     int64_t site, double* xi, double magic) {
  site_noise(q == 27 ? 27 : 19, kT, tau, rho, seed, step, (long)site, xi, magic);
}

void or_site_normals_n(const uint32_t* seed, int64_t step, int64_t site, int32_t ncalls, double* z) {
  site_normals(seed, step, (long)site, z, ncalls);
}

// D3Q27 basis: e[k * 27 + i] = e_k(c_i), b[k] = sum_i w_i e_k(c_i)^2, odd[k] = parity
void or_mode_basis27(double* e, double* b, int32_t* odd) {
  for (int k = 0; k < 27; ++k) {
    for (int i = 0; i < 27; ++i) e[k * 27 + i] = mode27_poly(k, CV[i]);
    b[k] = mode27_norm(k);
    odd[k] = mode27_odd(k) ? 1 : 0;
  }
}

// Velocities c[Q][3] and weights w[Q] of the set with q = 19 or 27; 1 for any other q.
int or_velocity_set_q(int32_t q, int32_t* c, double* w) {
  if (q != 19 && q != 27) return 1;
  for (int i = 0; i < q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = CV[i][a];
    w[i] = wq(q, i);
  }
  return 0;
}

void or_velocity_set(int32_t* c, double* w) { or_velocity_set_q(19, c, w); }

// Deviation equilibrium g_eq_i(delta rho, u) around rest density rho0.
void or_equilibrium_q(int32_t q, double rho0, double drho, const double* u, double* out) {
  equilibrium_dev<double>(q == 27 ? 27 : 19, drho, rho0 + drho, u, out);
}

void or_equilibrium(double rho0, double drho, const double* u, double* out) {
  or_equilibrium_q(19, rho0, drho, u, out);
}

// One Guo-forced collision at a single node: BGK (magic = 0) or two relaxation times.
void or_collide_node_q(int32_t q, double tau, double magic, double rho0, const double* g,
                       const double* F, double* out) {
  collide_node<double>(q == 27 ? 27 : 19, tau, rho0, g, F, out, magic);
}

void or_collide_node(double tau, double rho0, const double* g, const double* F, double* out) {
  or_collide_node_q(19, tau, 0.0, rho0, g, F, out);
}

void or_collide_node_trt(double tau, double magic, double rho0, const double* g, const double* F,
                         double* out) {
  or_collide_node_q(19, tau, magic, rho0, g, F, out);
}

// Streaming of a [Q][S] population array (post-collision in, pre-collision out).
void or_stream_q(int32_t q, const int32_t* L, const double* post, double* pre) {
  Model<double> m;
  set_geometry(q == 27 ? 27 : 19, L, m);
  std::vector<double> in, out((size_t)m.Q * m.P);
  load_pops(m, post, in);
  stream(m, in, out);
  store_pops(m, out, pre);
}

void or_stream(const int32_t* L, const double* post, double* pre) { or_stream_q(19, L, post, pre); }

// Trilinear interpolation of a [3][S] field at n positions.
void or_interpolate(const int32_t* L, const double* field, int32_t n, const double* X, double* U) {
  int Li[3] = {L[0], L[1], L[2]};
  long S = (long)L[0] * L[1] * L[2];
  std::vector<double> f(field, field + 3 * S);
  interpolate(Li, S, f, n, X, U);
}

// Trilinear spreading: field += sum_a W(X_a) F_a (the field is accumulated into).
void or_spread(const int32_t* L, int32_t n, const double* X, const double* F, double* field) {
  int Li[3] = {L[0], L[1], L[2]};
  long S = (long)L[0] * L[1] * L[2];
  std::vector<double> f(field, field + 3 * S);
  spread(Li, S, n, X, F, f);
  std::memcpy(field, f.data(), sizeof(double) * 3 * S);
}

// Stand-in force field and its energy at unwrapped positions X.
void or_forces(const or_params* p, const double* X, const double* X0, const int32_t* bonds,
               double* F) {
  Model<double> m;
  build_model<double>(p, X0, bonds, nullptr, m);
  std::vector<double> Xv(X, X + 3 * (size_t)p->n_atoms), Fv(3 * (size_t)p->n_atoms);
  atom_forces(m, Xv, Fv);
  std::memcpy(F, Fv.data(), sizeof(double) * 3 * p->n_atoms);
}

// The same force field evaluated atom by atom over cell-list candidates (the form the coupled
// step uses); equal to or_forces bit for bit.
void or_forces_by_atom(const or_params* p, const double* X, const double* X0, const int32_t* bonds,
                       double* F) {
  Model<double> m;
  build_model<double>(p, X0, bonds, nullptr, m);
  std::vector<double> Xv(X, X + 3 * (size_t)p->n_atoms), Fv(3 * (size_t)p->n_atoms);
  atom_forces_by_atom(m, Xv, Fv);
  std::memcpy(F, Fv.data(), sizeof(double) * 3 * p->n_atoms);
}

double or_energy(const or_params* p, const double* X, const double* X0, const int32_t* bonds) {
  Model<double> m;
  build_model<double>(p, X0, bonds, nullptr, m);
  std::vector<double> Xv(X, X + 3 * (size_t)p->n_atoms);
  return atom_energy(m, Xv);
}

// External force density field [3][S] for the given body-force kind.
void or_external_force(const or_params* p, const double* field, double* out) {
  long S = (long)p->L[0] * p->L[1] * p->L[2];
  std::vector<double> f;
  external_force<double>(p, field, f, S);
  std::memcpy(out, f.data(), sizeof(double) * 3 * S);
}

// Observables of the pre-collision state: rho = rho0 + sum g, u = (j + F_ext/2) / rho.
void or_observables(const or_params* p, const double* g, const double* field, double* rho,
                    double* u) {
  Model<double> m;
  set_geometry(q_of(p), p->L, m);
  std::vector<double> fext;
  external_force<double>(p, field, fext, m.S);
  std::vector<double> gv;
  load_pops(m, g, gv);
  for (long x = 0; x < m.S; ++x) {
    double dr, j[3];
    moments_at(m, gv, x, dr, j);
    double r = p->rho0 + dr;
    rho[x] = r;
    for (int c = 0; c < 3; ++c) u[c * m.S + x] = (j[c] + 0.5 * fext[c * m.S + x]) / r;
  }
}

// Conserved sums: [0] mass = sum_x (rho0 + sum_i g_i), [1..3] fluid momentum sum_x j,
// [4..6] atom momentum sum_a m v_a.
void or_invariants(const or_params* p, const double* g, const double* V, double* out) {
  long S = (long)p->L[0] * p->L[1] * p->L[2];
  for (int k = 0; k < 7; ++k) out[k] = 0.0;
  double dm = 0.0;   // sum of deviations, kept apart from the (large) rest mass
  const int Q = q_of(p);
  for (long x = 0; x < S; ++x) {
    for (int i = 0; i < Q; ++i) {
      double gi = g[i * S + x];
      dm += gi;
      for (int a = 0; a < 3; ++a) out[1 + a] += CV[i][a] * gi;
    }
  }
  out[0] = p->rho0 * (double)S + dm;
  for (int a = 0; a < p->n_atoms; ++a)
    for (int c = 0; c < 3; ++c) out[4 + c] += p->mass * V[3 * a + c];
}

// n_steps coupled steps in float64, in place on (g, X, V).  X0 are the tether anchors,
// field the [3][S] body force (bf_kind 3 only, else may be NULL).
int or_run(const or_params* p, double* g, double* X, double* V, const double* X0,
           const int32_t* bonds, const double* field, int32_t n_steps) {
  return run_impl<double>(p, g, X, V, X0, bonds, field, n_steps);
}

// Same scheme evaluated in float32 arithmetic (inputs/outputs still float64 arrays).
int or_run_f32(const or_params* p, double* g, double* X, double* V, const double* X0,
               const int32_t* bonds, const double* field, int32_t n_steps) {
  return run_impl<float>(p, g, X, V, X0, bonds, field, n_steps);
}

// Loss L = (1/N) sum_a |X_a(T) - (X_a(0) + D)|^2 after n_steps from (g, X, V), and its
// exact derivative along one direction by forward-mode dual numbers:
//   wrt = 0: d/d gamma;  wrt = 1: d/d tau;  wrt = 2: d/d eps of F_ext = field + eps * dfield
//   (bf_kind must be 3 for wrt = 2).
int or_loss_derivative(const or_params* p, const double* g, const double* X, const double* V,
                       const double* X0, const int32_t* bonds, const double* field,
                       const double* D, int32_t n_steps, int32_t wrt, const double* dfield,
                       double* loss, double* dloss) {
  if (!params_ok(p)) return 2;
  Model<Dual> m;
  build_model<Dual>(p, X0, bonds, field, m);
  if (wrt == 0) m.gamma = Dual(p->gamma, 1.0);
  else if (wrt == 1) m.tau = Dual(p->tau, 1.0);
  else if (wrt == 2) {
    if (p->bf_kind != 3 || !dfield) return 1;
    for (long k = 0; k < 3 * m.S; ++k) m.fext[k].d = dfield[k];
  } else {
    return 1;
  }
  State<Dual> s;
  s.step = p->step0;
  load_pops(m, g, s.g);
  s.X.resize(3 * (size_t)m.n_atoms);
  s.V.resize(3 * (size_t)m.n_atoms);
  for (long k = 0; k < 3L * m.n_atoms; ++k) {
    s.X[k] = Dual(X[k]);
    s.V[k] = Dual(V[k]);
  }
  Work<Dual> w;
  w.size(m);
  for (int n = 0; n < n_steps; ++n) coupled_step(m, s, w);
  Dual acc(0.0);
  for (int a = 0; a < m.n_atoms; ++a)
    for (int c = 0; c < 3; ++c) {
      Dual e = s.X[3 * a + c] - Dual(X[3 * a + c] + D[c]);
      acc += e * e;
    }
  acc = acc / Dual((double)m.n_atoms);
  *loss = acc.v;
  *dloss = acc.d;
  return 0;
}

// One coupled step from (g, X, V), with the outputs evaluated only where asked: the
// post-step pre-collision populations g'[k][0..Q-1] at sites site_idx[k], and X', V' of atoms
// atom_idx[k].  Same algorithm as or_run; the collision is evaluated only at the Q
// upstream nodes of each requested site, the force field only for requested atoms.
int or_step_sampled(const or_params* p, const double* g, const double* X, const double* V,
                    const double* X0, const int32_t* bonds, const double* field,
                    int32_t n_sites, const int64_t* site_idx, double* g_out,
                    int32_t n_idx, const int32_t* atom_idx, double* X_out, double* V_out) {
  if (!params_ok(p)) return 2;
  Model<double> m;
  build_model<double>(p, X0, bonds, field, m);
  State<double> s;
  s.step = p->step0;
  load_pops(m, g, s.g);
  s.X.assign(X, X + 3 * (size_t)m.n_atoms);
  s.V.assign(V, V + 3 * (size_t)m.n_atoms);
  Work<double> w;
  w.size(m);
  coupling_forces(m, s, w);
  const std::vector<double>& Fc = w.Fc;
  const std::vector<double>& Ftot = w.Ftot;
  const int* L = m.L;
  for (int k = 0; k < n_sites; ++k) {
    long xs = site_idx[k];
    long x = xs % L[0], y = (xs / L[0]) % L[1], z = xs / ((long)L[0] * L[1]);
    for (int i = 0; i < m.Q; ++i) {
      long src = site_index(L, wrap(x - CV[i][0], L[0]), wrap(y - CV[i][1], L[1]), wrap(z - CV[i][2], L[2]));
      double gin[QMAX], gout[QMAX], F[3];
      for (int q = 0; q < m.Q; ++q) gin[q] = s.g[q * m.P + src];
      for (int c = 0; c < 3; ++c) F[c] = Ftot[c * m.S + src];
      collide_node(m.Q, m.tau, m.rho0, gin, F, gout, m.trt_magic);
      if (m.kT > 0.0) {
        double rho = val(m.rho0);
        for (int q = 0; q < m.Q; ++q) rho += gin[q];
        double xi[QMAX];
        site_noise(m.Q, m.kT, val(m.tau), rho, m.seed, s.step, src, xi, m.trt_magic);
        gout[i] += xi[i];
      }
      g_out[(long)m.Q * k + i] = gout[i];
    }
  }
  for (int k = 0; k < n_idx; ++k) {
    int a = atom_idx[k];
    double F[3];
    atom_force_one(m, s.X, a, F);
    for (int c = 0; c < 3; ++c) {
      double v = s.V[3 * a + c] + (F[c] + Fc[3 * a + c]) / m.mass;
      V_out[3 * k + c] = v;
      X_out[3 * k + c] = s.X[3 * a + c] + v;
    }
  }
  return 0;
}

// Loss only, float64 (for central finite differences).
int or_loss(const or_params* p, const double* g, const double* X, const double* V,
            const double* X0, const int32_t* bonds, const double* field, const double* D,
            int32_t n_steps, double* loss) {
  if (!params_ok(p)) return 2;
  std::vector<double> gv(g, g + q_of(p) * (size_t)p->L[0] * p->L[1] * p->L[2]);
  std::vector<double> Xv(X, X + 3 * (size_t)p->n_atoms), Vv(V, V + 3 * (size_t)p->n_atoms);
  run_impl<double>(p, gv.data(), Xv.data(), Vv.data(), X0, bonds, field, n_steps);
  double acc = 0.0;
  for (int a = 0; a < p->n_atoms; ++a)
    for (int c = 0; c < 3; ++c) {
      double e = Xv[3 * a + c] - (X[3 * a + c] + D[c]);
      acc += e * e;
    }
  *loss = acc / p->n_atoms;
  return 0;
}

}  // extern "C"
