// Discrete adjoint of the coupled step (reverse mode), for gradients of a loss of the atoms'
// final state with respect to the friction gamma, the relaxation time tau and the external
// force-density field.
//
// The forward step n maps the stored post-collision buffer P^n, the atom positions X^n and
// velocities v^n to P^{n+1}, X^{n+1}, v^{n+1} (Section 2.2, Eqs. 1-3 and the friction
// coupling; see atoms.hip and lb_sweep.hip).  Its adjoint takes Lam^{n+1} = dL/dP^{n+1},
// lx = dL/dX^{n+1}, lv = dL/dv^{n+1} back to step n, accumulating dL/dgamma, dL/domega and
// dL/dF_ext on the way.  With h_i(x) = P^n_i(x - c_i) the pre-collision values at x and
// mu(x) = Lam^{n+1}(x) the adjoint of the collision output at x:
//   collision with Guo forcing, written as out = h + s - omega+ d+ - omega- d- with
//     d = h - geq(rho, u*) + s/2, u* = (j + F/2)/rho, s the Guo source before its prefactor
//     (BGK: omega- = omega+ = omega).  With nu_i = omega+ mu+_i + omega- mu-_i (mu+- the parts
//     of mu even and odd under c -> -c) and kappa = mu - nu/2:
//     a_i = mu_i - nu_i + l_rho + c_i . l_j      (l_j = l_u / rho,
//       l_rho = sum_i nu_i dgeq_i/drho - u*.l_u/rho,
//       l_u = sum_i [nu_i dgeq_i/du* + kappa_i ds_i/du*])
//     phi = dL/dF(x) = sum_i kappa_i ds_i/dF + l_u / (2 rho)
//     dL/domega+ += -sum_i mu+_i d_i,  dL/domega- += -sum_i mu-_i d_i
//   atoms (F_c = gamma (U - v), U = sum_k W_k u_c(node_k), the fluid gets -W_k F_c):
//     v'  = lv + lx                                       (X^{n+1} = X^n + v^{n+1})
//     lF_c = v'/m - sum_k W_k phi(node_k)
//     dL/dgamma += lF_c . (U - v);  l_U = gamma lF_c;  lv^n = v' - gamma lF_c
//     lx^n = lx + H_ff(X^n) v'/m + sum_k grad W_k [u_c(node_k) . l_U - F_c . phi(node_k)]
//   coupling velocity (u_c = (j + F_ext/2)/rho at nodes, from h):
//     l_uc(x) = sum_a W(X_a, x) l_U,a;  a_i += -u_c.l_uc/rho + c_i . l_uc/rho
//   and dL/dF_ext(x) += phi(x) + l_uc(x) / (2 rho)
//   thermal noise (kT > 0): out_i += A+ pe_i + A- po_i with A+- = sqrt(3 rho kT (2 omega+- -
//     omega+-^2)) and pe, po the step's fixed even and odd patterns, so
//     a_i += (sum mu pe A+ + sum mu po A-)/(2 rho) and
//     dL/domega+- += (sum mu p+-) A+- (1 - omega+-)/(2 omega+- - omega+-^2)
//   streaming (pull): Lam^n_i(x - c_i) = a_i(x), a push with one store per (i, x).
// The state of each step is recomputed from checkpoints by the host (lb_backward).
#include "atoms_common.h"

namespace lbmd {
namespace {

struct AdjLatticeArgs {
  const void* P;          // P^n (storage format)
  const float* lam_in;    // Lam^{n+1}, FP32 [Q][plane]
  float* lam_out;         // Lam^n
  long plane;
  int nx, ny, nz, S;
  float rho0, omega, omega_m;
  int bf_kind;
  const float* fext_tab;
  const float* fext_field;
  const uint32_t* tile_flag;
  const float* fcoup;     // spread coupling force of step n on flagged tiles
  float* fcoup_clear;     // the same buffer, cleared by the sweep (NULL in the tile pass)
  int* base_count;        // cleared by the sweep on flagged tiles
  const float* luc;       // dL/du_c on flagged tiles
  float* phi;             // out (tile pass): dL/dF on flagged tiles
  float* db;              // dL/dF_ext accumulated, [3][S], or NULL
  double* dom_part;       // per workgroup: partial dL/domega+ and dL/domega- [2][nblocks]
  const int* hot_list;
  const int* hot_count;
  float kT;               // thermal noise of the forward step (0: none)
  uint32_t seed0, seed1;
  int64_t step;
  FastDiv dnx, dny;
  int narrow;             // the FP32 Lam planes (and so the population planes) take 32-bit byte offsets
};

// Adjoint of the collision at one site (Q = 19 or 27 velocities): from mu (adjoint of the
// output) and the site's pre-collision values g and force F, the adjoint of g (in place of
// mu), phi = dL/dF, and this site's dL/domega+ and dL/domega- terms.  Also returns rho and the
// moments for the caller.
template <int Q>
__device__ __forceinline__ void collide_adjoint(float mu[Q], const float g[Q], float Fx, float Fy,
                                                float Fz, float rho0, float omega_p, float omega_m,
                                                float& phx, float& phy, float& phz, float& dom_p,
                                                float& dom_m, float& rho, float& jx, float& jy,
                                                float& jz) {
  float drho;
  moments<Q>(g, drho, jx, jy, jz);
  rho = rho0 + drho;
  const float inv = 1.0f / rho;
  const float ux = (jx + 0.5f * Fx) * inv;
  const float uy = (jy + 0.5f * Fy) * inv;
  const float uz = (jz + 0.5f * Fz) * inv;
  const float uu = ux * ux + uy * uy + uz * uz;
  const float uF = ux * Fx + uy * Fy + uz * Fz;
  const float ca = 0.5f * (omega_p + omega_m), cb = 0.5f * (omega_p - omega_m);
  float lrho_e = 0.f, lux = 0.f, luy = 0.f, luz = 0.f, lfx = 0.f, lfy = 0.f, lfz = 0.f;
  dom_p = dom_m = 0.f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const float cu = cdot<0>(ux, uy, uz, CX[i], CY[i], CZ[i]);
    const float cF = cdot<0>(Fx, Fy, Fz, CX[i], CY[i], CZ[i]);
    const float n = ca * mu[i] + cb * mu[OPP(i)];
    const float k = mu[i] - 0.5f * n;
    const float geq = wq<Q>(i) * (drho + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
    const float si = wq<Q>(i) * (3.0f * (cF - uF) + 9.0f * cu * cF);
    const float d = g[i] - geq + 0.5f * si;
    dom_p -= 0.5f * (mu[i] + mu[OPP(i)]) * d;
    dom_m -= 0.5f * (mu[i] - mu[OPP(i)]) * d;
    const float An = n * wq<Q>(i), Ak = k * wq<Q>(i);
    lrho_e += An * (1.0f + 3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
    // d geq_i / d u*: w rho (3 c + 9 cu c - 3 u);  d s_i / d u*: w (9 cF c - 3 F)
    const float kc = rho * (3.0f + 9.0f * cu);
    lux += An * (kc * (float)CX[i] - 3.0f * rho * ux) + Ak * (9.0f * cF * (float)CX[i] - 3.0f * Fx);
    luy += An * (kc * (float)CY[i] - 3.0f * rho * uy) + Ak * (9.0f * cF * (float)CY[i] - 3.0f * Fy);
    luz += An * (kc * (float)CZ[i] - 3.0f * rho * uz) + Ak * (9.0f * cF * (float)CZ[i] - 3.0f * Fz);
    // d s_i / d F (explicit): w (3 (c - u) + 9 cu c)
    const float kfc = 3.0f + 9.0f * cu;
    lfx += Ak * (kfc * (float)CX[i] - 3.0f * ux);
    lfy += Ak * (kfc * (float)CY[i] - 3.0f * uy);
    lfz += Ak * (kfc * (float)CZ[i] - 3.0f * uz);
  }
  const float ljx = lux * inv, ljy = luy * inv, ljz = luz * inv;
  const float lrho = lrho_e - (ux * lux + uy * luy + uz * luz) * inv;
  phx = lfx + 0.5f * ljx;
  phy = lfy + 0.5f * ljy;
  phz = lfz + 0.5f * ljz;
  // a_i = mu_i - nu_i + l_rho + c_i . l_j, nu recomputed from the old mu of i and its
  // opposite, so each opposite pair is updated together
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    if (i != 0 && (i & 1) == 0) continue;
    const int o = OPP(i);
    const float mi = mu[i], mo = mu[o];
    mu[i] = mi - (ca * mi + cb * mo) + lrho + cdot<0>(ljx, ljy, ljz, CX[i], CY[i], CZ[i]);
    if (o != i) mu[o] = mo - (ca * mo + cb * mi) + lrho + cdot<0>(ljx, ljy, ljz, CX[o], CY[o], CZ[o]);
  }
}

// per-site work shared by the tile pass and the sweep
template <int ST, int Q>
__device__ __forceinline__ void adj_site(const AdjLatticeArgs& a, int s, bool hot, bool sweep,
                                         float& dom_p, float& dom_m) {
  using T = typename Store<ST>::T;
  int x, y, z;
  site_xyz(s, a.nx, a.ny, a.dnx, a.dny, x, y, z);
  float g[Q], mu[Q];
  const bool narrow = a.narrow != 0;
  gather<ST, Q>(reinterpret_cast<const T*>(a.P), a.plane, x, y, z, a.nx, a.ny, a.nz, narrow, g);
  if (narrow) {
#pragma unroll
    for (int i = 0; i < Q; ++i) mu[i] = *plane_at(a.lam_in, i, a.plane, 4u * (uint32_t)s);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) mu[i] = a.lam_in[(size_t)i * a.plane + s];
  }
  float Ex, Ey, Ez;
  external_force(a.bf_kind, a.fext_tab, a.fext_field, a.plane, s, y, Ex, Ey, Ez);
  float Fx = Ex, Fy = Ey, Fz = Ez;
  if (hot) {
    Fx += a.fcoup[s];
    Fy += a.fcoup[a.plane + s];
    Fz += a.fcoup[2 * a.plane + s];
  }
  // the noise does not depend on F, so only the sweep needs its terms
  const bool noise = sweep && a.kT > 0.f;
  float mpe = 0.f, mpo = 0.f;   // sum_i mu_i pe_i, sum_i mu_i po_i of the noise patterns
  if (noise) {
    float pe[Q], po[Q];
    noise_patterns<Q>(a.seed0, a.seed1, a.step, s, pe, po);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      mpe += mu[i] * pe[i];
      mpo += mu[i] * po[i];
    }
  }
  float phx, phy, phz, rho, jx, jy, jz;
  collide_adjoint<Q>(mu, g, Fx, Fy, Fz, a.rho0, a.omega, a.omega_m, phx, phy, phz, dom_p, dom_m, rho,
                     jx, jy, jz);
  if (noise) {
    const float Ap = noise_amp(a.kT, rho, a.omega), Am = noise_amp(a.kT, rho, a.omega_m);
    const float lr = (mpe * Ap + mpo * Am) / (2.0f * rho);
#pragma unroll
    for (int i = 0; i < Q; ++i) mu[i] += lr;
    dom_p += mpe * Ap * (1.0f - a.omega) / (a.omega * (2.0f - a.omega));
    dom_m += mpo * Am * (1.0f - a.omega_m) / (a.omega_m * (2.0f - a.omega_m));
  }
  if (!sweep) {
    a.phi[s] = phx;
    a.phi[a.plane + s] = phy;
    a.phi[2 * a.plane + s] = phz;
    return;
  }
  float dbx = phx, dby = phy, dbz = phz;
  if (hot) {
    // the coupling velocity u_c = (j + F_ext/2)/rho read at this node by the atoms
    const float inv = 1.0f / rho;
    const float lx = a.luc[s] * inv, ly = a.luc[a.plane + s] * inv, lz = a.luc[2 * a.plane + s] * inv;
    const float ucx = (jx + 0.5f * Ex) * inv, ucy = (jy + 0.5f * Ey) * inv, ucz = (jz + 0.5f * Ez) * inv;
    const float lr = -(ucx * lx + ucy * ly + ucz * lz);
#pragma unroll
    for (int i = 0; i < Q; ++i) mu[i] += lr + cdot<0>(lx, ly, lz, CX[i], CY[i], CZ[i]);
    dbx += 0.5f * lx;
    dby += 0.5f * ly;
    dbz += 0.5f * lz;
    a.fcoup_clear[s] = 0.f;
    a.fcoup_clear[a.plane + s] = 0.f;
    a.fcoup_clear[2 * a.plane + s] = 0.f;
    a.base_count[s] = 0;
  }
  if (a.db) {
    a.db[s] += dbx;
    a.db[a.S + s] += dby;
    a.db[2 * a.S + s] += dbz;
  }
  // adjoint of the pull: the value read from (x - c_i) receives a_i
  const int xm = x == 0 ? a.nx - 1 : x - 1, xp = x == a.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? a.ny - 1 : y - 1, yp = y == a.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? a.nz - 1 : z - 1, zp = z == a.nz - 1 ? 0 : z + 1;
  const int nxy = a.nx * a.ny;
  if (narrow) {
    const uint32_t X3[3] = {4u * xm, 4u * x, 4u * xp};
    const uint32_t Y3[3] = {4u * a.nx * ym, 4u * a.nx * y, 4u * a.nx * yp};
    const uint32_t Z3[3] = {4u * nxy * zm, 4u * nxy * z, 4u * nxy * zp};
#pragma unroll
    for (int i = 0; i < Q; ++i)
      *plane_at(a.lam_out, i, a.plane, X3[1 - CX[i]] + Y3[1 - CY[i]] + Z3[1 - CZ[i]]) = mu[i];
  } else {
    const int X3[3] = {xm, x, xp};
    const int Y3[3] = {ym * a.nx, y * a.nx, yp * a.nx};
    const int Z3[3] = {zm * nxy, z * nxy, zp * nxy};
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const int dst = X3[1 - CX[i]] + Y3[1 - CY[i]] + Z3[1 - CZ[i]];
      a.lam_out[(size_t)i * a.plane + dst] = mu[i];
    }
  }
}

// FP64 sum of one value per thread over a 256-thread workgroup, in a fixed order
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[4];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (part[0] + part[1]) + (part[2] + part[3]);
  __syncthreads();
  return r;
}

// dL/dF at every site of the flagged tiles (one wavefront per tile)
template <int ST, int Q>
__global__ __launch_bounds__(256) void k_adj_tiles(AdjLatticeArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6, nwave = gridDim.x * 4;
  const int n = *a.hot_count;
  for (int k = wave; k < n; k += nwave) {
    const int s = (a.hot_list[k] << kTileShift) + lane;
    float dp, dm;
    if (s < a.S) adj_site<ST, Q>(a, s, true, false, dp, dm);
  }
}

// the adjoint sweep over all sites
template <int ST, int Q>
__global__ __launch_bounds__(kSweepBlock) void k_adj_sweep(AdjLatticeArgs a) {
  const int s = blockIdx.x * kSweepBlock + threadIdx.x;
  float dp = 0.f, dm = 0.f;
  if (s < a.S) {
    const bool hot = a.tile_flag != nullptr && a.tile_flag[s >> kTileShift] != 0u;
    adj_site<ST, Q>(a, s, hot, true, dp, dm);
  }
  const double bp = block_sum((double)dp);
  const double bm = block_sum((double)dm);
  if (threadIdx.x == 0) {
    a.dom_part[blockIdx.x] = bp;
    a.dom_part[gridDim.x + blockIdx.x] = bm;
  }
}

// ---- atoms ------------------------------------------------------------------------------------
struct AdjAtomArgs {
  int N;
  int n[3];
  long plane;
  float gamma, inv_mass;
  const float* x0;
  const float* d;     // [2][N][3] hi, lo
  const float* v;     // [2][N][3] hi, lo
  const float* fc;
  const float* U;
  const float* uc;
  const float* phi;
  const float* lx_in;
  const float* lv_in;
  float* lxa;         // out: the coupling's part of dL/dX^n (added to lx_out by k_adj_addx)
  float* lv_out;
  float* lU;
  float4* lf;         // k_adj_dir: v'/m per atom
  double* dg_part;    // per workgroup: partial dL/dgamma
};

__global__ __launch_bounds__(256) void k_adj_dir(AdjAtomArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.N) return;
  a.lf[i] = make_float4((a.lv_in[3 * i] + a.lx_in[3 * i]) * a.inv_mass,
                        (a.lv_in[3 * i + 1] + a.lx_in[3 * i + 1]) * a.inv_mass,
                        (a.lv_in[3 * i + 2] + a.lx_in[3 * i + 2]) * a.inv_mass, 0.f);
}

__global__ __launch_bounds__(256) void k_adj_atoms(AdjAtomArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  double dg = 0.0;
  if (i < a.N) {
    int i0[3];
    float fr[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      split(a.x0[3 * i + c], a.d[3 * i + c], a.d[3 * a.N + 3 * i + c], a.n[c], i0[c], fr[c]);
    const float fcx = a.fc[3 * i], fcy = a.fc[3 * i + 1], fcz = a.fc[3 * i + 2];
    float wpx = 0.f, wpy = 0.f, wpz = 0.f;    // sum W phi
    float gx = 0.f, gy = 0.f, gz = 0.f;       // -sum grad W (F_c . phi)
    float M[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};  // sum grad W u_c^T
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
      const int x = dx ? (i0[0] + 1 == a.n[0] ? 0 : i0[0] + 1) : i0[0];
      const int y = dy ? (i0[1] + 1 == a.n[1] ? 0 : i0[1] + 1) : i0[1];
      const int z = dz ? (i0[2] + 1 == a.n[2] ? 0 : i0[2] + 1) : i0[2];
      const int node = x + a.n[0] * (y + a.n[1] * z);
      const float wx = dx ? fr[0] : 1.0f - fr[0];
      const float wy = dy ? fr[1] : 1.0f - fr[1];
      const float wz = dz ? fr[2] : 1.0f - fr[2];
      const float w = wx * wy * wz;
      const float gw[3] = {(dx ? 1.f : -1.f) * wy * wz, (dy ? 1.f : -1.f) * wx * wz,
                           (dz ? 1.f : -1.f) * wx * wy};
      const float px = a.phi[node], py = a.phi[a.plane + node], pz = a.phi[2 * a.plane + node];
      const float ux = a.uc[node], uy = a.uc[a.plane + node], uz = a.uc[2 * a.plane + node];
      wpx += w * px;
      wpy += w * py;
      wpz += w * pz;
      const float fp = fcx * px + fcy * py + fcz * pz;
      gx -= gw[0] * fp;
      gy -= gw[1] * fp;
      gz -= gw[2] * fp;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        M[r][0] += gw[r] * ux;
        M[r][1] += gw[r] * uy;
        M[r][2] += gw[r] * uz;
      }
    }
    float vp[3], lfc[3], lu[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) vp[c] = a.lv_in[3 * i + c] + a.lx_in[3 * i + c];
    lfc[0] = vp[0] * a.inv_mass - wpx;
    lfc[1] = vp[1] * a.inv_mass - wpy;
    lfc[2] = vp[2] * a.inv_mass - wpz;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dg += (double)lfc[c] * (double)((a.U[3 * i + c] - a.v[3 * i + c]) - a.v[3 * a.N + 3 * i + c]);
      lu[c] = a.gamma * lfc[c];
      a.lU[3 * i + c] = lu[c];
      a.lv_out[3 * i + c] = vp[c] - lu[c];
    }
    a.lxa[3 * i] = gx + M[0][0] * lu[0] + M[0][1] * lu[1] + M[0][2] * lu[2];
    a.lxa[3 * i + 1] = gy + M[1][0] * lu[0] + M[1][1] * lu[1] + M[1][2] * lu[2];
    a.lxa[3 * i + 2] = gz + M[2][0] * lu[0] + M[2][1] * lu[1] + M[2][2] * lu[2];
  }
  const double b = block_sum(dg);
  if (threadIdx.x == 0) a.dg_part[blockIdx.x] = b;
}

// dL/dX^n = (dL/dX^{n+1} + H v'/m, the force field's Hessian-vector product) + the coupling's
// part (k_adj_atoms), one value per thread
__global__ __launch_bounds__(256) void k_adj_addx(float* lx_out, const float* lxa, int n3) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j < n3) lx_out[j] += lxa[j];
}

// dL/du_c at every site of the flagged tiles: the transpose of the interpolation applied to
// l_U, gathered over the base-node lists like the forward spread.  The entries of each list
// are taken in atom-index order, so the FP32 sum does not depend on binning order.
struct AdjSpreadArgs {
  int S;
  int n[3];
  long plane;
  const int* occ_tiles;
  const int* occ_count;
  const int* base_count;
  const int* base_list;
  const float4* atom_frac;
  const float* lU;
  float* luc;
};

__global__ __launch_bounds__(256) void k_adj_spread(AdjSpreadArgs a) {
  const int lane = threadIdx.x & 63;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6, nwave = gridDim.x * 4;
  const int ntile = *a.occ_count;
  for (int kt = wave; kt < ntile; kt += nwave) {
    const int s = (a.occ_tiles[kt] << kTileShift) + lane;
    if (s >= a.S) continue;
    const int x = s % nx;
    const int t = s / nx;
    const int y = t % ny;
    const int z = t / ny;
    // the 8 candidate base nodes; counts and first two list entries loaded up front
    int base[8], nb[8], e0[8], e1[8];
    bool few = true;   // every base node lists at most two atoms
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
      const int bx = dx ? (x == 0 ? nx - 1 : x - 1) : x;
      const int by = dy ? (y == 0 ? ny - 1 : y - 1) : y;
      const int bz = dz ? (z == 0 ? nz - 1 : z - 1) : z;
      base[k] = bx + nx * (by + ny * bz);
      const int c = a.base_count[base[k]];
      nb[k] = c > kBaseCap ? kBaseCap : c;
      e0[k] = a.base_list[(size_t)base[k] * kBaseCap];
      e1[k] = a.base_list[(size_t)base[k] * kBaseCap + 1];
      few = few && c <= 2;
    }
    // FP32 sums in a fixed order that depends only on the lists' contents (their order comes
    // from atomics): with at most two atoms per base node, the lower atom index of every
    // corner (corners in order), then the higher; otherwise corner by corner, atoms in
    // ascending index order.
    float sx = 0.f, sy = 0.f, sz = 0.f;
    auto term = [&](int k, int at, const float4& fr, float lx, float ly, float lz) {
      const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
      const float w = (dx ? fr.x : 1.0f - fr.x) * (dy ? fr.y : 1.0f - fr.y) * (dz ? fr.z : 1.0f - fr.z);
      sx += w * lx;
      sy += w * ly;
      sz += w * lz;
    };
    if (few) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (nb[k] == 2 && e1[k] < e0[k]) {
          const int t0 = e0[k];
          e0[k] = e1[k];
          e1[k] = t0;
        }
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        float4 fr[8];
        float l[8][3];
#pragma unroll
        for (int k = 0; k < 8; ++k) {   // a corner without entry q reads atom 0, unused
          const int at = nb[k] > q ? (q ? e1[k] : e0[k]) : 0;
          fr[k] = a.atom_frac[at];
          l[k][0] = a.lU[3 * at];
          l[k][1] = a.lU[3 * at + 1];
          l[k][2] = a.lU[3 * at + 2];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (nb[k] > q) term(k, 0, fr[k], l[k][0], l[k][1], l[k][2]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int n = nb[k];
        int ids[kBaseCap];
        for (int q = 0; q < n; ++q) {
          // insertion into the sorted prefix
          int v = a.base_list[(size_t)base[k] * kBaseCap + q], r = q;
          while (r > 0 && ids[r - 1] > v) {
            ids[r] = ids[r - 1];
            --r;
          }
          ids[r] = v;
        }
        for (int q = 0; q < n; ++q) {
          const int at = ids[q];
          term(k, at, a.atom_frac[at], a.lU[3 * at], a.lU[3 * at + 1], a.lU[3 * at + 2]);
        }
      }
    }
    a.luc[s] = sx;
    a.luc[a.plane + s] = sy;
    a.luc[2 * a.plane + s] = sz;
  }
}

// acc[0] += sum of the n0 partials p0; acc[1], acc[2] += sums of the two rows of n1 partials
// p1 (fixed order, one workgroup of kAdjRed threads).  Each thread keeps kAdjRedUnroll loads
// of each array in flight per round, so a large lattice's 65,536 sweep partials take a few
// memory round trips rather than one per element.
constexpr int kAdjRed = 1024, kAdjRedUnroll = 8;

__device__ __forceinline__ double block_sum_red(double v) {
  __shared__ double part[kAdjRed / 64];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < kAdjRed / 64; ++w) r += part[w];
  __syncthreads();
  return r;
}

// sum over k = threadIdx.x, + kAdjRed, ... < n of p[k], in that order
__device__ __forceinline__ double thread_sum(const double* p, int n) {
  double s = 0.0;
  for (int base = 0; base < n; base += kAdjRed * kAdjRedUnroll) {
    double v[kAdjRedUnroll];
#pragma unroll
    for (int u = 0; u < kAdjRedUnroll; ++u) {
      const int k = base + u * kAdjRed + (int)threadIdx.x;
      v[u] = k < n ? p[k] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kAdjRedUnroll; ++u) s += v[u];
  }
  return s;
}

__global__ __launch_bounds__(kAdjRed) void k_adj_reduce(const double* p0, int n0, const double* p1,
                                                        int n1, double* acc) {
  const double s0 = block_sum_red(thread_sum(p0, n0));
  const double s1 = block_sum_red(thread_sum(p1, n1));
  const double s2 = block_sum_red(thread_sum(p1 + n1, n1));
  if (threadIdx.x == 0) {
    acc[0] += s0;
    acc[1] += s1;
    acc[2] += s2;
  }
}

}  // namespace

// ---- launchers -------------------------------------------------------------------------------

static AdjLatticeArgs lattice_args(lb_ctx* c, const AdjointBuffers& b) {
  const Geometry& g = c->geo;
  const int par = (int)(c->step & 1);
  AdjLatticeArgs a;
  a.P = c->popbuf[c->cur];
  a.lam_in = b.lam_in;
  a.lam_out = b.lam_out;
  a.plane = g.plane;
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.S = (int)g.S;
  a.rho0 = c->p.rho0;
  a.omega = c->omega;
  a.omega_m = c->omega_m;
  a.bf_kind = c->p.bf_kind;
  a.fext_tab = (const float*)(c->ws + c->lay.fext_tab);
  a.fext_field = (const float*)(c->ws + c->lay.fext_field);
  a.tile_flag = (const uint32_t*)(c->bin + c->lay.tile_flag[par]);
  a.fcoup = (const float*)(c->bin + c->lay.fcoup[par]);
  a.fcoup_clear = (float*)(c->bin + c->lay.fcoup[par]);
  a.base_count = (int*)(c->bin + c->lay.base_count[par]);
  a.luc = b.luc;
  a.phi = b.phi;
  a.db = b.db;
  a.dom_part = b.dom_part;
  a.hot_list = (const int*)(c->bin + c->lay.occ_tiles[par]);
  a.hot_count = (const int*)(c->bin + c->lay.occ_count[par]) + 1;
  a.kT = c->p.kT;
  a.seed0 = c->p.seed[0];
  a.seed1 = c->p.seed[1];
  a.step = c->step;
  a.dnx = c->geo.div_nx;
  a.dny = c->geo.div_ny;
  // the Lam planes are FP32 whatever the storage format
  a.narrow = c->geo.narrow && (uint64_t)c->geo.S * 4u <= (1ull << 32) ? 1 : 0;
  return a;
}

static AdjAtomArgs atom_args(lb_ctx* c, const AdjointBuffers& b) {
  AdjAtomArgs a;
  a.N = c->p.n_atoms;
  a.n[0] = c->geo.nx;
  a.n[1] = c->geo.ny;
  a.n[2] = c->geo.nz;
  a.plane = c->geo.plane;
  a.gamma = c->p.gamma;
  a.inv_mass = 1.0f / c->p.mass;
  a.x0 = (const float*)(c->ws + c->lay.x0);
  a.d = (const float*)(c->ws + c->lay.disp[c->dcur]);
  a.v = (const float*)(c->ws + c->lay.vel);
  a.fc = (const float*)(c->bin + c->lay.fc);
  a.U = b.U;
  a.uc = (const float*)(c->bin + c->lay.uc);
  a.phi = b.phi;
  a.lx_in = b.lx_in;
  a.lv_in = b.lv_in;
  a.lxa = b.lxa;
  a.lv_out = b.lv_out;
  a.lU = b.lU;
  a.lf = b.lf;
  a.dg_part = b.dg_part;
  return a;
}

unsigned adjoint_atom_blocks(const lb_ctx* c) { return blocks(c->p.n_atoms, 256); }

hipError_t launch_adjoint_step(lb_ctx* c, const AdjointBuffers& b) {
  const Geometry& g = c->geo;
  const hipStream_t st = c->stream;
  const AdjAtomArgs aa = atom_args(c, b);
  const unsigned nab = adjoint_atom_blocks(c);
  // 1. direction v'/m and the force-field Hessian-vector product: lx_out = lx_in + H v'/m.  The
  // product needs only v'/m, the positions and the step's cell lists, and nothing after it
  // reads lx_out until k_adj_addx: with a side stream it runs there beside steps 2-6.
  hipLaunchKernelGGL(k_adj_dir, dim3(nab), dim3(256), 0, st, aa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool side = b.side != nullptr && b.side != st;
  if (side && ((e = hipEventRecord(b.ev_fork, st)) != hipSuccess ||
               (e = hipStreamWaitEvent(b.side, b.ev_fork, 0)) != hipSuccess))
    return e;
  if ((e = launch_force_hvp(c, b.lf, b.lx_in, b.lx_out, side ? b.side : st)) != hipSuccess) return e;
  if (side && (e = hipEventRecord(b.ev_join, b.side)) != hipSuccess) return e;
  // 2. dL/dF on the flagged tiles
  const AdjLatticeArgs la = lattice_args(c, b);
  const dim3 tgrid(persistent_grid(g.ntiles)), blk(256);
  const bool q27 = g.q == 27;
  switch (c->p.storage) {
    case LB_STORE_F32:
      if (q27) hipLaunchKernelGGL((k_adj_tiles<LB_STORE_F32, 27>), tgrid, blk, 0, st, la);
      else hipLaunchKernelGGL((k_adj_tiles<LB_STORE_F32, 19>), tgrid, blk, 0, st, la);
      break;
    case LB_STORE_F16:
      if (q27) hipLaunchKernelGGL((k_adj_tiles<LB_STORE_F16, 27>), tgrid, blk, 0, st, la);
      else hipLaunchKernelGGL((k_adj_tiles<LB_STORE_F16, 19>), tgrid, blk, 0, st, la);
      break;
    default:
      if (q27) hipLaunchKernelGGL((k_adj_tiles<LB_STORE_BF16, 27>), tgrid, blk, 0, st, la);
      else hipLaunchKernelGGL((k_adj_tiles<LB_STORE_BF16, 19>), tgrid, blk, 0, st, la);
      break;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 3. atoms
  hipLaunchKernelGGL(k_adj_atoms, dim3(nab), dim3(256), 0, st, aa);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 4. dL/du_c on the flagged tiles
  AdjSpreadArgs sa;
  const int par = (int)(c->step & 1);
  sa.S = (int)g.S;
  sa.n[0] = g.nx;
  sa.n[1] = g.ny;
  sa.n[2] = g.nz;
  sa.plane = g.plane;
  sa.occ_tiles = (const int*)(c->bin + c->lay.occ_tiles[par]);
  sa.occ_count = (const int*)(c->bin + c->lay.occ_count[par]) + 1;
  sa.base_count = (const int*)(c->bin + c->lay.base_count[par]);
  sa.base_list = (const int*)(c->bin + c->lay.base_list[par]);
  sa.atom_frac = (const float4*)(c->bin + c->lay.atom_frac);
  sa.lU = b.lU;
  sa.luc = b.luc;
  hipLaunchKernelGGL(k_adj_spread, tgrid, blk, 0, st, sa);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 5. the adjoint sweep
  const dim3 sgrid(g.nblocks), sblk(kSweepBlock);
  switch (c->p.storage) {
    case LB_STORE_F32:
      if (q27) hipLaunchKernelGGL((k_adj_sweep<LB_STORE_F32, 27>), sgrid, sblk, 0, st, la);
      else hipLaunchKernelGGL((k_adj_sweep<LB_STORE_F32, 19>), sgrid, sblk, 0, st, la);
      break;
    case LB_STORE_F16:
      if (q27) hipLaunchKernelGGL((k_adj_sweep<LB_STORE_F16, 27>), sgrid, sblk, 0, st, la);
      else hipLaunchKernelGGL((k_adj_sweep<LB_STORE_F16, 19>), sgrid, sblk, 0, st, la);
      break;
    default:
      if (q27) hipLaunchKernelGGL((k_adj_sweep<LB_STORE_BF16, 27>), sgrid, sblk, 0, st, la);
      else hipLaunchKernelGGL((k_adj_sweep<LB_STORE_BF16, 19>), sgrid, sblk, 0, st, la);
      break;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 6. FP64 accumulators
  hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(kAdjRed), 0, st, (const double*)b.dg_part, (int)nab,
                     (const double*)b.dom_part, g.nblocks, b.acc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // 7. dL/dX^n: the product (joined from the side stream) plus the coupling's part
  if (side && (e = hipStreamWaitEvent(st, b.ev_join, 0)) != hipSuccess) return e;
  const int n3 = 3 * c->p.n_atoms;
  hipLaunchKernelGGL(k_adj_addx, dim3(blocks(n3, 256)), dim3(256), 0, st, b.lx_out, (const float*)b.lxa, n3);
  return hipGetLastError();
}

}  // namespace lbmd
