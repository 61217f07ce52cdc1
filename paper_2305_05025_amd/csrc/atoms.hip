// Atom-side kernels for gfx950: friction coupling to the lattice and the stand-in force
// field.
//
// Coupling (paper Section 2.2, friction-coupling paragraph): the fluid velocity at an atom
// is the linear interpolation over its eight nearest nodes, the atom feels
// F_c = gamma (U - v), and the fluid receives -F_c through the forcing term with the same
// eight trilinear weights.  The fluid velocity at a node is u_c = (j + F_ext/2)/rho of the
// pre-collision state (Eqs. 2-3); the atoms' own force is not included.
//
// k_couple runs eight lanes per atom (one per stencil node): each lane pulls its node's 19
// pre-collision values, forms u_c and its weighted share; three xor-shuffles within the
// 8-lane group give U; every lane then adds its weighted share of -F_c to its node.  The
// deposit is a fixed-point (2^-40) 64-bit integer atomic add, so the summed force per node
// does not depend on the order in which atoms arrive.  The lane also raises the flag of
// the 256-site tile that holds its node, so the sweep reads the force field only there.
//
// Positions are kept as the caller's unwrapped anchors x0 plus a displacement d, so that
// pair vectors (x0_i - x0_j) + (d_i - d_j) and stencil fractions keep full FP32 precision
// at any box size.
#include "lbmd_internal.h"

namespace lbmd {
namespace {

struct CoupleArgs {
  const void* f;          // current population buffer
  int storage;
  long plane;
  int nx, ny, nz;
  float rho0, gamma;
  int bf_kind;
  const float* fext_tab;
  const float* fext_field;
  const float* x0;
  const float* d;
  const float* v;
  float* fc;              // out: friction force on each atom
  long long* fcoup;       // [3][plane] fixed point
  uint32_t* tile_flag;
  int N;
  // neighbour-list binning (nc[0] == 0 when off)
  int nc[3];
  float inv_cw[3];
  int* cell_count;
  int* cell_atoms;
  uint32_t* err;
};

__device__ __forceinline__ float load_pop(const void* f, int storage, size_t idx) {
  if (storage == LB_STORE_F32) return reinterpret_cast<const float*>(f)[idx];
  if (storage == LB_STORE_F16) return (float)reinterpret_cast<const _Float16*>(f)[idx];
  return __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(f)[idx] << 16);
}

__device__ __forceinline__ int wrapi(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// integer cell and fraction of (x0 + d) along one axis, with the integer part wrapped
// (the clamp keeps a diverging displacement, which the velocity check reports, from
// producing out-of-range integer conversions)
__device__ __forceinline__ void split(float x0, float d, int n, int& i0, float& frac) {
  const float ia = floorf(x0);
  const float t = fminf(fmaxf((x0 - ia) + d, -1.0e6f), 1.0e6f);
  const float fl = floorf(t);
  frac = t - fl;
  i0 = wrapi((int)ia + (int)fl, n);
}

// value * 2^40 rounded to an integer; clamped so that a diverging state (which the velocity
// check reports) cannot overflow the conversion
__device__ __forceinline__ long long to_fixed(float v) {
  float q = rintf(v * kFixScale);
  q = fminf(fmaxf(q, -4.0e18f), 4.0e18f);
  return (long long)q;
}

__global__ __launch_bounds__(256) void k_couple(CoupleArgs a) {
  const int tid = blockIdx.x * 256 + threadIdx.x;
  const int atom = tid >> 3;
  const int k = tid & 7;
  const bool valid = atom < a.N;
  const int at = valid ? atom : a.N - 1;
  int i0[3];
  float fr[3];
  const int n3[3] = {a.nx, a.ny, a.nz};
#pragma unroll
  for (int c = 0; c < 3; ++c) split(a.x0[3 * at + c], a.d[3 * at + c], n3[c], i0[c], fr[c]);
  const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
  const int x = dx ? (i0[0] + 1 == a.nx ? 0 : i0[0] + 1) : i0[0];
  const int y = dy ? (i0[1] + 1 == a.ny ? 0 : i0[1] + 1) : i0[1];
  const int z = dz ? (i0[2] + 1 == a.nz ? 0 : i0[2] + 1) : i0[2];
  const float w = (dx ? fr[0] : 1.0f - fr[0]) * (dy ? fr[1] : 1.0f - fr[1]) *
                  (dz ? fr[2] : 1.0f - fr[2]);
  // pre-collision values at the node, pulled from its upstream neighbours
  const int xm = x == 0 ? a.nx - 1 : x - 1, xp = x == a.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? a.ny - 1 : y - 1, yp = y == a.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? a.nz - 1 : z - 1, zp = z == a.nz - 1 ? 0 : z + 1;
  const int nxy = a.nx * a.ny;
  const int X3[3] = {xm, x, xp};
  const int Y3[3] = {ym * a.nx, y * a.nx, yp * a.nx};
  const int Z3[3] = {zm * nxy, z * nxy, zp * nxy};
  float drho = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const int src = X3[1 - CX[i]] + Y3[1 - CY[i]] + Z3[1 - CZ[i]];
    const float gi = load_pop(a.f, a.storage, (size_t)i * a.plane + src);
    drho += gi;
    if (CX[i] == 1) jx += gi;
    if (CX[i] == -1) jx -= gi;
    if (CY[i] == 1) jy += gi;
    if (CY[i] == -1) jy -= gi;
    if (CZ[i] == 1) jz += gi;
    if (CZ[i] == -1) jz -= gi;
  }
  const int node = x + a.nx * y + nxy * z;
  float Fx = 0.f, Fy = 0.f, Fz = 0.f;
  if (a.bf_kind == LB_BF_KOLMOGOROV || a.bf_kind == LB_BF_SIGN_SHEAR) {
    Fx = a.fext_tab[y];
  } else if (a.bf_kind == LB_BF_FIELD) {
    Fx = a.fext_field[node];
    Fy = a.fext_field[a.plane + node];
    Fz = a.fext_field[2 * a.plane + node];
  }
  const float inv = 1.0f / (a.rho0 + drho);
  float Ux = w * ((jx + 0.5f * Fx) * inv);
  float Uy = w * ((jy + 0.5f * Fy) * inv);
  float Uz = w * ((jz + 0.5f * Fz) * inv);
  // sum over the 8 lanes of this atom (lanes 8a..8a+7 of the wavefront)
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) {
    Ux += __shfl_xor(Ux, o, 64);
    Uy += __shfl_xor(Uy, o, 64);
    Uz += __shfl_xor(Uz, o, 64);
  }
  if (!valid) return;
  const float fcx = a.gamma * (Ux - a.v[3 * atom]);
  const float fcy = a.gamma * (Uy - a.v[3 * atom + 1]);
  const float fcz = a.gamma * (Uz - a.v[3 * atom + 2]);
  // the fluid receives -F_c with the interpolation weights
  const long long qx = to_fixed(-w * fcx);
  const long long qy = to_fixed(-w * fcy);
  const long long qz = to_fixed(-w * fcz);
  unsigned long long* fq = reinterpret_cast<unsigned long long*>(a.fcoup);
  if (qx) atomicAdd(fq + node, (unsigned long long)qx);
  if (qy) atomicAdd(fq + a.plane + node, (unsigned long long)qy);
  if (qz) atomicAdd(fq + 2 * a.plane + node, (unsigned long long)qz);
  a.tile_flag[node >> kTileShift] = 1u;
  if (k == 0) {
    a.fc[3 * atom] = fcx;
    a.fc[3 * atom + 1] = fcy;
    a.fc[3 * atom + 2] = fcz;
    if (a.nc[0] > 0) {
      int cc[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float Y = (float)i0[c] + fr[c];
        int q = (int)(Y * a.inv_cw[c]);
        cc[c] = q >= a.nc[c] ? a.nc[c] - 1 : q;
      }
      const int cell = cc[0] + a.nc[0] * (cc[1] + a.nc[1] * cc[2]);
      const int slot = atomicAdd(a.cell_count + cell, 1);
      if (slot < kCellCap)
        a.cell_atoms[(size_t)cell * kCellCap + slot] = atom;
      else
        atomicOr(a.err, kErrOverflow);
    }
  }
}

// Order each cell's atoms by index, so that the pair sums below run in a fixed order and
// the whole step is bitwise reproducible.
__global__ __launch_bounds__(256) void k_cell_sort(int* count, int* atoms, long ncell) {
  const long c = blockIdx.x * 256L + threadIdx.x;
  if (c >= ncell) return;
  int n = count[c];
  if (n > kCellCap) n = kCellCap;
  int* p = atoms + c * kCellCap;
  for (int i = 1; i < n; ++i) {
    const int v = p[i];
    int j = i - 1;
    while (j >= 0 && p[j] > v) {
      p[j + 1] = p[j];
      --j;
    }
    p[j + 1] = v;
  }
}

struct ForceArgs {
  int N;
  float L[3], invL[3];
  const float* x0;
  const float* d;       // X^n - x0
  float* d_next;        // X^{n+1} - x0
  float* v;             // in/out
  const float* fc;
  float inv_mass;
  float k_tether;
  const int* bond_off;
  const int* bond_nbr;
  float k_bond, r0_bond;
  float lj_eps24, lj_sigma2, lj_rc2;
  int lj_exclude_bonded;
  int nc[3];
  float inv_cw[3];
  const int* cell_count;
  const int* cell_atoms;
  uint32_t* err;
};

__device__ __forceinline__ float min_image(float r, float L, float invL) {
  return r - L * rintf(r * invL);
}

__global__ __launch_bounds__(256) void k_forces_integrate(ForceArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.N) return;
  const float xi = a.x0[3 * i], yi = a.x0[3 * i + 1], zi = a.x0[3 * i + 2];
  const float dxi = a.d[3 * i], dyi = a.d[3 * i + 1], dzi = a.d[3 * i + 2];
  float Fx = -a.k_tether * dxi, Fy = -a.k_tether * dyi, Fz = -a.k_tether * dzi;
  const int b0 = a.bond_off[i], b1 = a.bond_off[i + 1];
  for (int b = b0; b < b1; ++b) {
    const int j = a.bond_nbr[b];
    const float rx = min_image((xi - a.x0[3 * j]) + (dxi - a.d[3 * j]), a.L[0], a.invL[0]);
    const float ry = min_image((yi - a.x0[3 * j + 1]) + (dyi - a.d[3 * j + 1]), a.L[1], a.invL[1]);
    const float rz = min_image((zi - a.x0[3 * j + 2]) + (dzi - a.d[3 * j + 2]), a.L[2], a.invL[2]);
    const float rl = sqrtf(rx * rx + ry * ry + rz * rz);
    const float f = -a.k_bond * (rl - a.r0_bond) / rl;
    Fx += f * rx;
    Fy += f * ry;
    Fz += f * rz;
  }
  if (a.nc[0] > 0) {
    // the atom's own cell, from its wrapped position
    int cc[3];
    const float xs[3] = {xi, yi, zi}, ds[3] = {dxi, dyi, dzi};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      int i0;
      float fr;
      split(xs[c], ds[c], (int)a.L[c], i0, fr);
      const float Y = (float)i0 + fr;
      const int q = (int)(Y * a.inv_cw[c]);
      cc[c] = q >= a.nc[c] ? a.nc[c] - 1 : q;
    }
    for (int oz = -1; oz <= 1; ++oz) {
      int cz = cc[2] + oz;
      cz = cz < 0 ? cz + a.nc[2] : (cz >= a.nc[2] ? cz - a.nc[2] : cz);
      for (int oy = -1; oy <= 1; ++oy) {
        int cy = cc[1] + oy;
        cy = cy < 0 ? cy + a.nc[1] : (cy >= a.nc[1] ? cy - a.nc[1] : cy);
        for (int ox = -1; ox <= 1; ++ox) {
          int cx = cc[0] + ox;
          cx = cx < 0 ? cx + a.nc[0] : (cx >= a.nc[0] ? cx - a.nc[0] : cx);
          const long cell = cx + (long)a.nc[0] * (cy + (long)a.nc[1] * cz);
          int n = a.cell_count[cell];
          n = n > kCellCap ? kCellCap : n;
          const int* list = a.cell_atoms + cell * kCellCap;
          for (int q = 0; q < n; ++q) {
            const int j = list[q];
            if (j == i) continue;
            const float rx = min_image((xi - a.x0[3 * j]) + (dxi - a.d[3 * j]), a.L[0], a.invL[0]);
            const float ry = min_image((yi - a.x0[3 * j + 1]) + (dyi - a.d[3 * j + 1]), a.L[1], a.invL[1]);
            const float rz = min_image((zi - a.x0[3 * j + 2]) + (dzi - a.d[3 * j + 2]), a.L[2], a.invL[2]);
            const float r2 = rx * rx + ry * ry + rz * rz;
            if (!(r2 < a.lj_rc2)) continue;
            if (a.lj_exclude_bonded) {
              bool bonded = false;
              for (int b = b0; b < b1; ++b) bonded = bonded || (a.bond_nbr[b] == j);
              if (bonded) continue;
            }
            const float inv2 = 1.0f / r2;
            const float sr2 = a.lj_sigma2 * inv2;
            const float sr6 = sr2 * sr2 * sr2;
            const float f = a.lj_eps24 * (2.0f * sr6 * sr6 - sr6) * inv2;
            Fx += f * rx;
            Fy += f * ry;
            Fz += f * rz;
          }
        }
      }
    }
  }
  // symplectic Euler: v^{n+1} = v^n + (F_ff + F_c)/m, X^{n+1} = X^n + v^{n+1}
  const float vx = a.v[3 * i] + (Fx + a.fc[3 * i]) * a.inv_mass;
  const float vy = a.v[3 * i + 1] + (Fy + a.fc[3 * i + 1]) * a.inv_mass;
  const float vz = a.v[3 * i + 2] + (Fz + a.fc[3 * i + 2]) * a.inv_mass;
  if (!__builtin_isfinite(vx + vy + vz)) atomicOr(a.err, kErrNonFinite);
  a.v[3 * i] = vx;
  a.v[3 * i + 1] = vy;
  a.v[3 * i + 2] = vz;
  a.d_next[3 * i] = dxi + vx;
  a.d_next[3 * i + 1] = dyi + vy;
  a.d_next[3 * i + 2] = dzi + vz;
}

struct PrepArgs {
  int* cell_count;
  long ncell;
  uint32_t* tile_flag;
  int ntiles;
};

__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
  const long t = blockIdx.x * 256L + threadIdx.x;
  if (t < a.ncell) a.cell_count[t] = 0;
  if (t < a.ntiles) a.tile_flag[t] = 0u;
}

__global__ __launch_bounds__(256) void k_read_atoms(int N, const float* x0, const float* d,
                                                    const float* v, float* xo, float* vo) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= 3 * N) return;
  if (xo) xo[t] = x0[t] + d[t];
  if (vo) vo[t] = v[t];
}

}  // namespace

hipError_t launch_prep(lb_ctx* c) {
  PrepArgs a;
  a.cell_count = (int*)(c->ws + c->lay.cell_count);
  a.ncell = c->geo.ncell;
  a.tile_flag = (uint32_t*)(c->ws + c->lay.tile_flag);
  a.ntiles = c->geo.ntiles;
  const long n = a.ncell > a.ntiles ? a.ncell : a.ntiles;
  hipLaunchKernelGGL(k_prep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, a);
  return hipGetLastError();
}

hipError_t launch_couple(lb_ctx* c) {
  const Geometry& g = c->geo;
  CoupleArgs a;
  a.f = c->ws + c->lay.pop[c->cur];
  a.storage = c->p.storage;
  a.plane = g.plane;
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.rho0 = c->p.rho0;
  a.gamma = c->p.gamma;
  a.bf_kind = c->p.bf_kind;
  a.fext_tab = (const float*)(c->ws + c->lay.fext_tab);
  a.fext_field = (const float*)(c->ws + c->lay.fext_field);
  a.x0 = (const float*)(c->ws + c->lay.x0);
  a.d = (const float*)(c->ws + c->lay.disp[c->dcur]);
  a.v = (const float*)(c->ws + c->lay.vel);
  a.fc = (float*)(c->ws + c->lay.fc);
  a.fcoup = (long long*)(c->ws + c->lay.fcoup);
  a.tile_flag = (uint32_t*)(c->ws + c->lay.tile_flag);
  a.N = c->p.n_atoms;
  for (int k = 0; k < 3; ++k) {
    a.nc[k] = g.nc[k];
    a.inv_cw[k] = g.inv_cw[k];
  }
  a.cell_count = (int*)(c->ws + c->lay.cell_count);
  a.cell_atoms = (int*)(c->ws + c->lay.cell_atoms);
  a.err = (uint32_t*)(c->ws + c->lay.err);
  const long threads = 8L * a.N;
  hipLaunchKernelGGL(k_couple, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, c->stream, a);
  return hipGetLastError();
}

hipError_t launch_cell_sort(lb_ctx* c) {
  const long n = c->geo.ncell;
  hipLaunchKernelGGL(k_cell_sort, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                     (int*)(c->ws + c->lay.cell_count), (int*)(c->ws + c->lay.cell_atoms), n);
  return hipGetLastError();
}

hipError_t launch_forces_integrate(lb_ctx* c) {
  const Geometry& g = c->geo;
  ForceArgs a;
  a.N = c->p.n_atoms;
  const int n3[3] = {g.nx, g.ny, g.nz};
  for (int k = 0; k < 3; ++k) {
    a.L[k] = (float)n3[k];
    a.invL[k] = 1.0f / (float)n3[k];
    a.nc[k] = g.nc[k];
    a.inv_cw[k] = g.inv_cw[k];
  }
  a.x0 = (const float*)(c->ws + c->lay.x0);
  a.d = (const float*)(c->ws + c->lay.disp[c->dcur]);
  a.d_next = (float*)(c->ws + c->lay.disp[c->dcur ^ 1]);
  a.v = (float*)(c->ws + c->lay.vel);
  a.fc = (const float*)(c->ws + c->lay.fc);
  a.inv_mass = 1.0f / c->p.mass;
  a.k_tether = c->p.k_tether;
  a.bond_off = (const int*)(c->ws + c->lay.bond_off);
  a.bond_nbr = (const int*)(c->ws + c->lay.bond_nbr);
  a.k_bond = c->p.k_bond;
  a.r0_bond = c->p.r0_bond;
  a.lj_eps24 = 24.0f * c->p.lj_eps;
  a.lj_sigma2 = c->p.lj_sigma * c->p.lj_sigma;
  a.lj_rc2 = c->p.lj_rc * c->p.lj_rc;
  a.lj_exclude_bonded = c->p.lj_exclude_bonded;
  a.cell_count = (const int*)(c->ws + c->lay.cell_count);
  a.cell_atoms = (const int*)(c->ws + c->lay.cell_atoms);
  a.err = (uint32_t*)(c->ws + c->lay.err);
  hipLaunchKernelGGL(k_forces_integrate, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0,
                     c->stream, a);
  return hipGetLastError();
}

hipError_t launch_read_atoms(lb_ctx* c, float* x, float* v) {
  const int N = c->p.n_atoms;
  hipLaunchKernelGGL(k_read_atoms, dim3((unsigned)((3L * N + 255) / 256)), dim3(256), 0, c->stream,
                     N, (const float*)(c->ws + c->lay.x0),
                     (const float*)(c->ws + c->lay.disp[c->dcur]),
                     (const float*)(c->ws + c->lay.vel), x, v);
  return hipGetLastError();
}

}  // namespace lbmd
