// Lattice kernels for gfx950: the fused pull-stream + BGK/Guo collision sweep, readback of
// the moments, and the FP64 conservation sums.
//
// Eq. (1) of the paper (Section 2.2), written for deviations g_i = f_i - w_i rho0 and read
// with the standard BGK sign (relaxation toward equilibrium):
//   g_i(x + c_i, t + 1) = g_i - omega (g_i - g_i^eq) + S_i
// with omega = 1/tau, the second-order equilibrium, the moments of Eqs. (2)-(3), and the
// forcing term S_i in the Guo form (velocity shifted by F/2, prefactor 1 - omega/2).
//
// Layout: populations are Q planes (structure of arrays) of `plane` elements, Q = 19 (D3Q19)
// or 27 (D3Q27), site index s = x + nx (y + ny z).  The stored buffer holds post-collision
// values at the site that produced them; a site's pre-collision values are pulled from its Q
// upstream neighbours
// (x - c_i), so every load of a wavefront is a contiguous (possibly 4-byte shifted) run and
// every store is a full aligned run.  The sweep reads buffer A and writes buffer B.
//
// One thread per site, 256 sites per workgroup.  A workgroup is also the unit ("tile") of
// the sparse atom force: tiles that atoms touched in this step carry a flag, and only their
// sites read (and clear) the fixed-point coupling-force field.
#include <mutex>
#include <type_traits>

#include "atoms_common.h"

namespace lbmd {
namespace {

struct SweepArgs {
  const void* fin;
  void* fout;
  long plane;
  int nx, ny, nz, S;
  float rho0, omega, pref;
  int bf_kind;
  const float* fext_tab;
  const float* fext_field;
  const uint32_t* tile_flag;   // NULL when there are no atoms
  float* fcoup;                // [3][plane] spread coupling force (hot tiles only)
  int* base_count;             // [plane] cleared here for hot tiles, with fcoup (NULL: both kept)
  uint32_t* err;
  float kT;                    // thermal noise (NOISE instances only)
  uint32_t seed0, seed1;
  int64_t step;
  float omega_m;               // rate of the odd part (TRT instances only)
  FastDiv dnx, dny;
  int narrow;                  // planes take 32-bit byte offsets
  // Non-temporal population loads: every stored value is read exactly once per sweep, and
  // when a workgroup's sites are whole rows (nx divides kSweepBlock) its x-shifted reads share
  // no cache line with another workgroup's, so keeping the lines would only displace the data
  // of the kernels that run beside the sweep.  Rows that straddle workgroups (which run on
  // different XCDs) share a line at each boundary, and a line not kept is then fetched twice.
  int nt_loads;
};

// The update of site s = (x, y, z): pull its pre-collision values, add the coupling force
// (Fcx, Fcy, Fcz) to the external force density when `coupled`, collide (BGK or two relaxation
// times, Guo forcing), add the thermal noise, store.  Q velocities (19 or 27).
template <int ST, bool NOISE, bool TRT, int Q>
__device__ __forceinline__ void update_site(const SweepArgs& a, int s, int x, int y, int z,
                                            bool coupled, float Fcx, float Fcy, float Fcz) {
  using T = typename Store<ST>::T;
  float g[Q];
  if (a.nt_loads)
    gather<ST, Q, true>(reinterpret_cast<const T*>(a.fin), a.plane, x, y, z, a.nx, a.ny, a.nz,
                        a.narrow != 0, g);
  else
    gather<ST, Q, false>(reinterpret_cast<const T*>(a.fin), a.plane, x, y, z, a.nx, a.ny, a.nz,
                         a.narrow != 0, g);
  float Fx, Fy, Fz;
  external_force(a.bf_kind, a.fext_tab, a.fext_field, a.plane, s, y, Fx, Fy, Fz);
  if (coupled) {
    Fx += Fcx;
    Fy += Fcy;
    Fz += Fcz;
  }
  float rho = 0.f;
  if constexpr (NOISE) {
    rho = a.rho0;
#pragma unroll
    for (int i = 0; i < Q; ++i) rho += g[i];
  }
  bool ok;
  if constexpr (TRT) ok = collide_trt<Q>(g, Fx, Fy, Fz, a.rho0, a.omega, a.omega_m);
  else ok = collide<Q>(g, Fx, Fy, Fz, a.rho0, a.omega, a.pref);
  if (!ok) atomicOr(a.err, kErrNonFinite);
  if constexpr (NOISE) {
    float pe[Q], po[Q];
    noise_patterns<Q>(a.seed0, a.seed1, a.step, s, pe, po);
    const float Ap = noise_amp(a.kT, rho, a.omega);
    const float Am = TRT ? noise_amp(a.kT, rho, a.omega_m) : Ap;
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] += Ap * pe[i] + Am * po[i];
  }
  T* out = reinterpret_cast<T*>(a.fout);
  if (a.narrow) {
    const uint32_t so = (uint32_t)s * (uint32_t)sizeof(T);
#pragma unroll
    for (int i = 0; i < Q; ++i) Store<ST>::st(plane_at(out, i, a.plane, so), g[i]);
  } else {
#pragma unroll
    for (int i = 0; i < Q; ++i) Store<ST>::st(out + (size_t)i * a.plane + s, g[i]);
  }
}

// Q velocities (19 or 27)
template <int ST, bool NOISE, bool TRT, int Q>
__device__ __forceinline__ void sweep_site(const SweepArgs& a, int s, bool hot) {
  int x, y, z;
  site_xyz(s, a.nx, a.ny, a.dnx, a.dny, x, y, z);
  float Fcx = 0.f, Fcy = 0.f, Fcz = 0.f;
  if (hot) {
    // atoms touched this 64-site tile: add their spread force and leave the per-step
    // atom-side buffers clear for the next step
    float* fc = a.fcoup;
    Fcx = fc[s];
    Fcy = fc[a.plane + s];
    Fcz = fc[2 * a.plane + s];
    if (a.base_count) {
      fc[s] = 0.f;
      fc[a.plane + s] = 0.f;
      fc[2 * a.plane + s] = 0.f;
      a.base_count[s] = 0;
    }
  }
  update_site<ST, NOISE, TRT, Q>(a, s, x, y, z, hot, Fcx, Fcy, Fcz);
}

// One thread per site, in site order.  The instances without noise are held to 64 VGPRs (8
// wavefronts per SIMD) except the D3Q27 TRT one, which would spill there.
template <int ST, bool NOISE, bool TRT, int Q>
__global__ __launch_bounds__(kSweepBlock)
__attribute__((amdgpu_waves_per_eu(NOISE || (TRT && Q == 27) ? 1 : 8))) void k_sweep(SweepArgs a) {
  const int s = blockIdx.x * kSweepBlock + threadIdx.x;
  if (s >= a.S) return;
  const bool hot = a.tile_flag != nullptr && a.tile_flag[s >> kTileShift] != 0u;
  sweep_site<ST, NOISE, TRT, Q>(a, s, hot);
}

// ---- the coupled sweep, fused -------------------------------------------------------------------
// The lattice is cut into bricks of 16 x 4 x 4 sites.  A hot brick (one that some atom's stencil
// touches) is handled by one workgroup, which does the whole coupling of Section 2.2 for it
// before updating its sites:
//   1. the atoms listed for the brick mark their 8 stencil nodes, which lie in the brick and a
//      one-node halo around it (18 x 6 x 6 nodes);
//   2. the coupling velocity u_c = (j + F_ext/2)/rho of the pre-collision state at every marked
//      node, pulled from the stored populations, into LDS;
//   3. per listed atom: U = trilinear interpolation of u_c at X^n, F_c = gamma (U - v); the
//      workgroup of the brick holding the atom's stencil base stores F_c for the integration;
//      -W F_c is added to the brick's own stencil nodes in an LDS force tile, in 2^-40 fixed
//      point (integer sums do not depend on the order of their terms);
//   4. every site of the brick: collision with F = F_ext + spread force, streaming, store.
// An atom near a brick face is listed in each brick its stencil reaches, and its F_c is then
// computed by each of them with the same instructions on the same values.  The arithmetic of
// u_c, U (summed over the corners in the order (0+1)+(2+3), (4+5)+(6+7), then the two halves),
// F_c and the spread is that of k_node_u, k_couple and k_spread, so the results are the same
// bits as the unfused kernels'.  The remaining sites are swept by k_sweep_cold.
struct HotArgs {
  int nb0, nb1;            // bricks along x and y
  const int* hot;          // the hot bricks, compacted
  const int* nhot;         // their number
  const int* brick_count;
  const int* brick_list;   // [nbricks][kBrickCap]
  int N;
  const float* x0;
  const float* d;          // [2][N][3]: hi, lo
  const float* v;          // [2][N][3]: hi, lo
  float gamma;
  float* fc;               // out: friction force on each atom
};

constexpr int kHotAtomsPerThread = (kBrickCap + kSweepBlock - 1) / kSweepBlock;

__device__ __forceinline__ int wrap_once(int r, int n) {
  r = r < 0 ? r + n : r;
  return r >= n ? r - n : r;
}

template <int ST, bool NOISE, bool TRT, int Q>
__global__ __launch_bounds__(kSweepBlock) void k_hot_sweep(SweepArgs a, HotArgs h) {
  using T = typename Store<ST>::T;
  __shared__ float ucx[kHaloNodes], ucy[kHaloNodes], ucz[kHaloNodes];
  __shared__ unsigned char need[kHaloNodes];
  __shared__ long long fsx[kSweepBlock], fsy[kSweepBlock], fsz[kSweepBlock];
  const int t = threadIdx.x;
  const int nhot = *h.nhot;
  // XCD x takes the x-th contiguous eighth of the list: neighbouring hot bricks share halo
  // nodes, which then meet in that XCD's L2 (the grid is a multiple of 8 workgroups)
  const int chunk = (nhot + 7) >> 3;
  const int k0 = (int)(blockIdx.x & 7u) * chunk, k1 = min(k0 + chunk, nhot);
  for (int k = k0 + (int)(blockIdx.x >> 3); k < k1; k += (int)(gridDim.x >> 3)) {
    const int b = h.hot[k];
    const int bx = b % h.nb0, byz = b / h.nb0;
    const int by = byz % h.nb1, bz = byz / h.nb1;
    const int ox = bx * kBrickX, oy = by * kBrickY, oz = bz * kBrickZ;   // brick origin
    for (int q = t; q < kHaloNodes; q += kSweepBlock) need[q] = 0;
    fsx[t] = 0;
    fsy[t] = 0;
    fsz[t] = 0;
    __syncthreads();
    // 1. listed atoms: stencil base relative to the halo's lower corner (ox - 1, oy - 1, oz - 1),
    //    wrapped once into the lattice.  The list holds the atoms whose stencil reaches the
    //    brick, so their relative base is at most 16, 4, 4 along x, y, z, and every node index
    //    below stays within the halo (and within the lattice after one wrap).
    const int na = min(h.brick_count[b], kBrickCap);
    int at[kHotAtomsPerThread], rel[kHotAtomsPerThread];
    float frs[kHotAtomsPerThread][3];
#pragma unroll
    for (int j = 0; j < kHotAtomsPerThread; ++j) {
      const int slot = t + j * kSweepBlock;
      at[j] = slot < na ? h.brick_list[(long)b * kBrickCap + slot] : -1;
    }
#pragma unroll
    for (int j = 0; j < kHotAtomsPerThread; ++j) {
      rel[j] = 0;
      frs[j][0] = frs[j][1] = frs[j][2] = 0.f;
      if (at[j] < 0) continue;
      const int i = at[j];
      int i0[3];
      split(h.x0[3 * i], h.d[3 * i], h.d[3 * h.N + 3 * i], a.nx, i0[0], frs[j][0]);
      split(h.x0[3 * i + 1], h.d[3 * i + 1], h.d[3 * h.N + 3 * i + 1], a.ny, i0[1], frs[j][1]);
      split(h.x0[3 * i + 2], h.d[3 * i + 2], h.d[3 * h.N + 3 * i + 2], a.nz, i0[2], frs[j][2]);
      const int rx = wrap_once(i0[0] - ox + 1, a.nx);
      const int ry = wrap_once(i0[1] - oy + 1, a.ny);
      const int rz = wrap_once(i0[2] - oz + 1, a.nz);
      rel[j] = rx + kHaloX * (ry + kHaloY * rz);
#pragma unroll
      for (int c = 0; c < 8; ++c)
        need[rel[j] + (c & 1) + kHaloX * (((c >> 1) & 1) + kHaloY * ((c >> 2) & 1))] = 1;
    }
    __syncthreads();
    // 2. u_c at the marked halo nodes
    for (int q = t; q < kHaloNodes; q += kSweepBlock) {
      if (!need[q]) continue;
      const int hx = q % kHaloX, hyz = q / kHaloX;
      const int x = wrap_once(ox - 1 + hx, a.nx);
      const int y = wrap_once(oy - 1 + hyz % kHaloY, a.ny);
      const int z = wrap_once(oz - 1 + hyz / kHaloY, a.nz);
      const int s = x + a.nx * (y + a.ny * z);
      float g[Q];
      gather<ST, Q>(reinterpret_cast<const T*>(a.fin), a.plane, x, y, z, a.nx, a.ny, a.nz,
                    a.narrow != 0, g);
      float drho, jx, jy, jz, Fx, Fy, Fz;
      moments<Q>(g, drho, jx, jy, jz);
      external_force(a.bf_kind, a.fext_tab, a.fext_field, a.plane, s, y, Fx, Fy, Fz);
      const float inv = 1.0f / (a.rho0 + drho);
      ucx[q] = (jx + 0.5f * Fx) * inv;
      ucy[q] = (jy + 0.5f * Fy) * inv;
      ucz[q] = (jz + 0.5f * Fz) * inv;
    }
    __syncthreads();
    // 3. friction of each listed atom; its spread onto this brick's nodes
#pragma unroll
    for (int j = 0; j < kHotAtomsPerThread; ++j) {
      if (at[j] < 0) continue;
      const int i = at[j];
      float wk[8], ux[8], uy[8], uz[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
        wk[c] = (dx ? frs[j][0] : 1.0f - frs[j][0]) * (dy ? frs[j][1] : 1.0f - frs[j][1]) *
                (dz ? frs[j][2] : 1.0f - frs[j][2]);
        const int q = rel[j] + dx + kHaloX * (dy + kHaloY * dz);
        ux[c] = wk[c] * ucx[q];
        uy[c] = wk[c] * ucy[q];
        uz[c] = wk[c] * ucz[q];
      }
      const float Ux = ((ux[0] + ux[1]) + (ux[2] + ux[3])) + ((ux[4] + ux[5]) + (ux[6] + ux[7]));
      const float Uy = ((uy[0] + uy[1]) + (uy[2] + uy[3])) + ((uy[4] + uy[5]) + (uy[6] + uy[7]));
      const float Uz = ((uz[0] + uz[1]) + (uz[2] + uz[3])) + ((uz[4] + uz[5]) + (uz[6] + uz[7]));
      const float* vlo = h.v + 3 * h.N;
      const float fx = h.gamma * ((Ux - h.v[3 * i]) - vlo[3 * i]);
      const float fy = h.gamma * ((Uy - h.v[3 * i + 1]) - vlo[3 * i + 1]);
      const float fz = h.gamma * ((Uz - h.v[3 * i + 2]) - vlo[3 * i + 2]);
      const int rx = rel[j] % kHaloX, ryz = rel[j] / kHaloX;
      const int ry = ryz % kHaloY, rz = ryz / kHaloY;
      // stencil base node and its brick: that brick's workgroup stores F_c
      const int b0x = wrap_once(ox - 1 + rx, a.nx), b0y = wrap_once(oy - 1 + ry, a.ny),
                b0z = wrap_once(oz - 1 + rz, a.nz);
      if ((b0x >> kBrickShiftX) == bx && (b0y >> kBrickShiftY) == by && (b0z >> kBrickShiftZ) == bz) {
        h.fc[3 * i] = fx;
        h.fc[3 * i + 1] = fy;
        h.fc[3 * i + 2] = fz;
      }
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
        const int lx = wrap_once(b0x + dx, a.nx) - ox;
        const int ly = wrap_once(b0y + dy, a.ny) - oy;
        const int lz = wrap_once(b0z + dz, a.nz) - oz;
        if (lx < 0 || lx >= kBrickX || ly < 0 || ly >= kBrickY || lz < 0 || lz >= kBrickZ) continue;
        const int l = lx + kBrickX * (ly + kBrickY * lz);
        atomicAdd(reinterpret_cast<unsigned long long*>(&fsx[l]), (unsigned long long)to_fixed(-wk[c] * fx, kFixScale));
        atomicAdd(reinterpret_cast<unsigned long long*>(&fsy[l]), (unsigned long long)to_fixed(-wk[c] * fy, kFixScale));
        atomicAdd(reinterpret_cast<unsigned long long*>(&fsz[l]), (unsigned long long)to_fixed(-wk[c] * fz, kFixScale));
      }
    }
    __syncthreads();
    // 4. the brick's sites
    const int x = ox + (t & (kBrickX - 1));
    const int y = oy + ((t >> kBrickShiftX) & (kBrickY - 1));
    const int z = oz + (t >> (kBrickShiftX + kBrickShiftY));
    if (x < a.nx && y < a.ny && z < a.nz)
      update_site<ST, NOISE, TRT, Q>(a, x + a.nx * (y + a.ny * z), x, y, z, true,
                                     (float)fsx[t] * kFixInv, (float)fsy[t] * kFixInv,
                                     (float)fsz[t] * kFixInv);
    __syncthreads();   // LDS is reused by the next brick
  }
}

// Every site outside the hot bricks: the plain stream-and-collide update.
template <int ST, bool NOISE, bool TRT, int Q>
__global__ __launch_bounds__(kSweepBlock)
__attribute__((amdgpu_waves_per_eu(NOISE || (TRT && Q == 27) ? 1 : 8))) void k_sweep_cold(
    SweepArgs a, const int* brick_count, int nb0, int nb1) {
  const int s = blockIdx.x * kSweepBlock + threadIdx.x;
  if (s >= a.S) return;
  int x, y, z;
  site_xyz(s, a.nx, a.ny, a.dnx, a.dny, x, y, z);
  if (brick_count[(x >> kBrickShiftX) + nb0 * ((y >> kBrickShiftY) + nb1 * (z >> kBrickShiftZ))] != 0)
    return;
  update_site<ST, NOISE, TRT, Q>(a, s, x, y, z, false, 0.f, 0.f, 0.f);
}

template <int ST>
void launch_sweep_st(int q, bool noise, bool trt, dim3 grid, dim3 block, hipStream_t st,
                     const SweepArgs& a) {
  if (q == 27) {
    if (noise && trt) hipLaunchKernelGGL((k_sweep<ST, true, true, 27>), grid, block, 0, st, a);
    else if (noise) hipLaunchKernelGGL((k_sweep<ST, true, false, 27>), grid, block, 0, st, a);
    else if (trt) hipLaunchKernelGGL((k_sweep<ST, false, true, 27>), grid, block, 0, st, a);
    else hipLaunchKernelGGL((k_sweep<ST, false, false, 27>), grid, block, 0, st, a);
  } else if (noise && trt) hipLaunchKernelGGL((k_sweep<ST, true, true, 19>), grid, block, 0, st, a);
  else if (noise) hipLaunchKernelGGL((k_sweep<ST, true, false, 19>), grid, block, 0, st, a);
  else if (trt) hipLaunchKernelGGL((k_sweep<ST, false, true, 19>), grid, block, 0, st, a);
  else hipLaunchKernelGGL((k_sweep<ST, false, false, 19>), grid, block, 0, st, a);
}

// Launch kernel template K<ST, Q> for the context's storage format and velocity set.
template <class F>
void dispatch_store_q(const lb_ctx* c, F&& launch) {
  const bool q27 = c->geo.q == 27;
  switch (c->p.storage) {
    case LB_STORE_F32:
      if (q27) launch(std::integral_constant<int, LB_STORE_F32>{}, std::integral_constant<int, 27>{});
      else launch(std::integral_constant<int, LB_STORE_F32>{}, std::integral_constant<int, 19>{});
      break;
    case LB_STORE_F16:
      if (q27) launch(std::integral_constant<int, LB_STORE_F16>{}, std::integral_constant<int, 27>{});
      else launch(std::integral_constant<int, LB_STORE_F16>{}, std::integral_constant<int, 19>{});
      break;
    default:
      if (q27) launch(std::integral_constant<int, LB_STORE_BF16>{}, std::integral_constant<int, 27>{});
      else launch(std::integral_constant<int, LB_STORE_BF16>{}, std::integral_constant<int, 19>{});
      break;
  }
}

// ---- readback -------------------------------------------------------------------------------
struct ReadArgs {
  const void* f;
  long plane;
  int nx, ny, nz, S;
  float rho0;
  int bf_kind;
  const float* fext_tab;
  const float* fext_field;
  float* rho;   // [S] or NULL
  float* u;     // [3][S] or NULL
  float* pops;  // [Q][S] or NULL
};

template <int ST, int Q>
__global__ __launch_bounds__(256) void k_read(ReadArgs a) {
  using T = typename Store<ST>::T;
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= a.S) return;
  const int x = s % a.nx;
  const int t = s / a.nx;
  const int y = t % a.ny;
  const int z = t / a.ny;
  float g[Q];
  gather<ST, Q>(reinterpret_cast<const T*>(a.f), a.plane, x, y, z, a.nx, a.ny, a.nz, false, g);
  if (a.pops) {
#pragma unroll
    for (int i = 0; i < Q; ++i) a.pops[(size_t)i * a.S + s] = g[i];
  }
  if (a.rho || a.u) {
    float drho, jx, jy, jz, Fx, Fy, Fz;
    moments<Q>(g, drho, jx, jy, jz);
    external_force(a.bf_kind, a.fext_tab, a.fext_field, a.plane, s, y, Fx, Fy, Fz);
    const float rho = a.rho0 + drho;
    if (a.rho) a.rho[s] = rho;
    if (a.u) {
      const float inv = 1.0f / rho;
      a.u[s] = (jx + 0.5f * Fx) * inv;
      a.u[(size_t)a.S + s] = (jy + 0.5f * Fy) * inv;
      a.u[2 * (size_t)a.S + s] = (jz + 0.5f * Fz) * inv;
    }
  }
}

// ---- state upload: the pull at y reads slot y - c_i, so g_i(x) is stored at x - c_i ----
struct WriteArgs {
  void* f;
  long plane;
  int nx, ny, nz, S;
  const float* pops;  // [Q][S]
};

template <int ST, int Q>
__global__ __launch_bounds__(256) void k_write(WriteArgs a) {
  using T = typename Store<ST>::T;
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= a.S) return;
  const int x = s % a.nx;
  const int t = s / a.nx;
  const int y = t % a.ny;
  const int z = t / a.ny;
  const int xm = x == 0 ? a.nx - 1 : x - 1, xp = x == a.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? a.ny - 1 : y - 1, yp = y == a.ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? a.nz - 1 : z - 1, zp = z == a.nz - 1 ? 0 : z + 1;
  const int nxy = a.nx * a.ny;
  const int X3[3] = {xm, x, xp};
  const int Y3[3] = {ym * a.nx, y * a.nx, yp * a.nx};
  const int Z3[3] = {zm * nxy, z * nxy, zp * nxy};
  T* f = reinterpret_cast<T*>(a.f);
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const int dst = X3[1 - CX[i]] + Y3[1 - CY[i]] + Z3[1 - CZ[i]];
    Store<ST>::st(f + (size_t)i * a.plane + dst, a.pops[(size_t)i * a.S + s]);
  }
}

// ---- FP64 conservation sums -------------------------------------------------------------------
// Streaming permutes values between sites, so the lattice totals of the stored buffer equal
// those of the pre-collision state; no gather is needed.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct RedArgs {
  const void* f;
  long plane;
  int S;
  double* partial;  // [kRedBlocks][4]
  uint32_t* err;
};

template <int ST, int Q>
__global__ __launch_bounds__(256) void k_reduce_pops(RedArgs a) {
  using T = typename Store<ST>::T;
  const T* f = reinterpret_cast<const T*>(a.f);
  double m = 0.0, px = 0.0, py = 0.0, pz = 0.0;
  bool finite = true;
  for (int s = blockIdx.x * 256 + threadIdx.x; s < a.S; s += gridDim.x * 256) {
    float g[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) g[i] = Store<ST>::ld(f + (size_t)i * a.plane + s);
    double dm = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const double gi = (double)g[i];
      dm += gi;
      if (CX[i] == 1) jx += gi;
      if (CX[i] == -1) jx -= gi;
      if (CY[i] == 1) jy += gi;
      if (CY[i] == -1) jy -= gi;
      if (CZ[i] == 1) jz += gi;
      if (CZ[i] == -1) jz -= gi;
    }
    finite = finite && __builtin_isfinite(dm + jx + jy + jz);
    m += dm;
    px += jx;
    py += jy;
    pz += jz;
  }
  if (!finite) atomicOr(a.err, kErrNonFinite);
  __shared__ double sh[4][4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  m = wave_sum(m);
  px = wave_sum(px);
  py = wave_sum(py);
  pz = wave_sum(pz);
  if (lane == 0) {
    sh[wid][0] = m;
    sh[wid][1] = px;
    sh[wid][2] = py;
    sh[wid][3] = pz;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    a.partial[blockIdx.x * 4 + k] = ((sh[0][k] + sh[1][k]) + sh[2][k]) + sh[3][k];
  }
}

struct FinalArgs {
  const double* partial;
  int nblocks;
  const float* vel;   // [2][N][3]: hi, lo
  int N;
  float mass;
  double rest_mass;   // rho0 * S
  double* out;        // [8]
  uint32_t* err;
};

__global__ __launch_bounds__(1024) void k_reduce_final(FinalArgs a) {
  __shared__ double sh[16][7];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < a.nblocks; b += 1024)
    for (int k = 0; k < 4; ++k) acc[k] += a.partial[b * 4 + k];
  bool finite = true;
  for (int i = threadIdx.x; i < a.N; i += 1024) {
    const float vx = a.vel[3 * i], vy = a.vel[3 * i + 1], vz = a.vel[3 * i + 2];
    const float* lo = a.vel + 3 * a.N;
    finite = finite && __builtin_isfinite(vx + vy + vz);
    acc[4] += (double)a.mass * ((double)vx + (double)lo[3 * i]);
    acc[5] += (double)a.mass * ((double)vy + (double)lo[3 * i + 1]);
    acc[6] += (double)a.mass * ((double)vz + (double)lo[3 * i + 2]);
  }
  if (!finite) atomicOr(a.err, kErrNonFinite);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < 7; ++k) {
    const double v = wave_sum(acc[k]);
    if (lane == 0) sh[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const int k = threadIdx.x;
    double v = 0.0;
    for (int w = 0; w < 16; ++w) v += sh[w][k];
    if (k == 0) v += a.rest_mass;
    a.out[k] = v;
  }
}

__global__ void k_zero(uint32_t* p, size_t n_words) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n_words;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// two equal-length word copies in one launch (the atoms' displacement and velocity)
__global__ void k_copy_pair(uint32_t* d0, const uint32_t* s0, uint32_t* d1, const uint32_t* s1,
                            size_t n_words) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < 2 * n_words;
       i += (size_t)gridDim.x * blockDim.x) {
    if (i < n_words)
      d0[i] = s0[i];
    else
      d1[i - n_words] = s1[i - n_words];
  }
}

__global__ void k_store_i64(int64_t* dst, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}

int blocks_for(long n, int per) { return (int)((n + per - 1) / per); }

}  // namespace

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  // every workspace region is a multiple of 4 bytes and 256-byte aligned
  const size_t words = bytes / 4;
  if (words == 0) return hipSuccess;
  int blocks = (int)((words + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, (uint32_t*)p, words);
  return hipGetLastError();
}

hipError_t launch_copy_pair(void* d0, const void* s0, void* d1, const void* s1, size_t bytes,
                            hipStream_t s) {
  // both regions are multiples of 4 bytes (FP32 arrays)
  const size_t words = bytes / 4;
  if (words == 0) return hipSuccess;
  int blocks = (int)((2 * words + 255) / 256);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_copy_pair, dim3(blocks), dim3(256), 0, s, (uint32_t*)d0, (const uint32_t*)s0,
                     (uint32_t*)d1, (const uint32_t*)s1, words);
  return hipGetLastError();
}

hipError_t launch_store_i64(void* dst, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_store_i64, dim3(1), dim3(64), 0, s, (int64_t*)dst, v);
  return hipGetLastError();
}

hipError_t launch_sweep(lb_ctx* c, const void* fin, void* fout, hipStream_t st) {
  const Geometry& g = c->geo;
  SweepArgs a;
  a.fin = fin;
  a.fout = fout;
  a.plane = g.plane;
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.S = (int)g.S;
  a.rho0 = c->p.rho0;
  a.omega = c->omega;
  a.pref = 1.0f - 0.5f * c->omega;
  a.bf_kind = c->p.bf_kind;
  a.fext_tab = (const float*)(c->ws + c->lay.fext_tab);
  a.fext_field = (const float*)(c->ws + c->lay.fext_field);
  const int par = (int)(c->step & 1);
  a.tile_flag = c->p.n_atoms > 0 ? (const uint32_t*)(c->bin + c->lay.tile_flag[par]) : nullptr;
  a.fcoup = (float*)(c->bin + c->lay.fcoup[par]);
  a.base_count = c->keep_coupling ? nullptr : (int*)(c->bin + c->lay.base_count[par]);
  a.err = (uint32_t*)(c->ws + c->lay.err);
  a.kT = c->p.kT;
  a.seed0 = c->p.seed[0];
  a.seed1 = c->p.seed[1];
  a.step = c->step;
  a.omega_m = c->omega_m;
  a.dnx = g.div_nx;
  a.dny = g.div_ny;
  a.narrow = g.narrow ? 1 : 0;
  a.nt_loads = kSweepBlock % g.nx == 0 ? 1 : 0;
  const dim3 block(kSweepBlock), grid(g.nblocks);
  const bool noise = c->p.kT > 0.0f, trt = c->p.trt_magic > 0.0f;
  switch (c->p.storage) {
    case LB_STORE_F32: launch_sweep_st<LB_STORE_F32>(g.q, noise, trt, grid, block, st, a); break;
    case LB_STORE_F16: launch_sweep_st<LB_STORE_F16>(g.q, noise, trt, grid, block, st, a); break;
    default: launch_sweep_st<LB_STORE_BF16>(g.q, noise, trt, grid, block, st, a); break;
  }
  return hipGetLastError();
}

namespace {

// Launch K<storage, noise, two relaxation times, Q> for the context's parameters.
template <class F>
void dispatch_sweep(const lb_ctx* c, F&& launch) {
  using std::integral_constant;
  const bool noise = c->p.kT > 0.0f, trt = c->p.trt_magic > 0.0f;
  dispatch_store_q(c, [&](auto st, auto q) {
    if (noise && trt) launch(st, integral_constant<bool, true>{}, integral_constant<bool, true>{}, q);
    else if (noise) launch(st, integral_constant<bool, true>{}, integral_constant<bool, false>{}, q);
    else if (trt) launch(st, integral_constant<bool, false>{}, integral_constant<bool, true>{}, q);
    else launch(st, integral_constant<bool, false>{}, integral_constant<bool, false>{}, q);
  });
}

SweepArgs sweep_args(lb_ctx* c, const void* fin, void* fout) {
  const Geometry& g = c->geo;
  SweepArgs a;
  a.fin = fin;
  a.fout = fout;
  a.plane = g.plane;
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.S = (int)g.S;
  a.rho0 = c->p.rho0;
  a.omega = c->omega;
  a.pref = 1.0f - 0.5f * c->omega;
  a.bf_kind = c->p.bf_kind;
  a.fext_tab = (const float*)(c->ws + c->lay.fext_tab);
  a.fext_field = (const float*)(c->ws + c->lay.fext_field);
  a.tile_flag = nullptr;
  a.fcoup = nullptr;
  a.base_count = nullptr;
  a.err = (uint32_t*)(c->ws + c->lay.err);
  a.kT = c->p.kT;
  a.seed0 = c->p.seed[0];
  a.seed1 = c->p.seed[1];
  a.step = c->step;
  a.omega_m = c->omega_m;
  a.dnx = g.div_nx;
  a.dny = g.div_ny;
  a.narrow = g.narrow ? 1 : 0;
  a.nt_loads = 0;   // hot bricks share lines at every brick face
  return a;
}

}  // namespace

// Workgroups of the hot-brick sweep: persistent over the list of hot bricks (at most one per
// brick and eight per atom), a multiple of 8, at most 2048 (eight per CU).
static unsigned hot_grid(const lb_ctx* c) {
  long n = std::min(c->geo.nbricks, 8L * c->p.n_atoms);
  if (n > 2048) n = 2048;
  return (unsigned)((std::max(n, 8L) + 7) & ~7L);
}

hipError_t launch_hot_sweep(lb_ctx* c, const void* fin, void* fout, hipStream_t st) {
  const SweepArgs a = sweep_args(c, fin, fout);
  const int par = (int)(c->step & 1);
  HotArgs h;
  h.nb0 = c->geo.nb[0];
  h.nb1 = c->geo.nb[1];
  h.hot = (const int*)(c->ws + c->lay.hot_bricks[par]);
  h.nhot = (const int*)(c->bin + c->lay.occ_count[par]) + 1;
  h.brick_count = (const int*)(c->ws + c->lay.brick_count[par]);
  h.brick_list = (const int*)(c->ws + c->lay.brick_list[par]);
  h.N = c->p.n_atoms;
  h.x0 = (const float*)(c->ws + c->lay.x0);
  h.d = (const float*)(c->ws + c->lay.disp[c->dcur]);
  h.v = (const float*)(c->ws + c->lay.vel);
  h.gamma = c->p.gamma;
  h.fc = (float*)(c->bin + c->lay.fc);
  const dim3 grid(hot_grid(c)), block(kSweepBlock);
  dispatch_sweep(c, [&](auto st_, auto nz, auto tr, auto q) {
    hipLaunchKernelGGL((k_hot_sweep<decltype(st_)::value, decltype(nz)::value, decltype(tr)::value,
                                    decltype(q)::value>),
                       grid, block, 0, st, a, h);
  });
  return hipGetLastError();
}

hipError_t launch_cold_sweep(lb_ctx* c, const void* fin, void* fout, hipStream_t st) {
  const SweepArgs a = sweep_args(c, fin, fout);
  const int par = (int)(c->step & 1);
  const int* bc = (const int*)(c->ws + c->lay.brick_count[par]);
  const int nb0 = c->geo.nb[0], nb1 = c->geo.nb[1];
  const dim3 grid(c->geo.nblocks), block(kSweepBlock);
  dispatch_sweep(c, [&](auto st_, auto nz, auto tr, auto q) {
    hipLaunchKernelGGL((k_sweep_cold<decltype(st_)::value, decltype(nz)::value, decltype(tr)::value,
                                     decltype(q)::value>),
                       grid, block, 0, st, a, bc, nb0, nb1);
  });
  return hipGetLastError();
}

static hipError_t launch_read(lb_ctx* c, float* rho, float* u, float* pops) {
  const Geometry& g = c->geo;
  ReadArgs a;
  a.f = c->popbuf[c->cur];
  a.plane = g.plane;
  a.nx = g.nx;
  a.ny = g.ny;
  a.nz = g.nz;
  a.S = (int)g.S;
  a.rho0 = c->p.rho0;
  a.bf_kind = c->p.bf_kind;
  a.fext_tab = (const float*)(c->ws + c->lay.fext_tab);
  a.fext_field = (const float*)(c->ws + c->lay.fext_field);
  a.rho = rho;
  a.u = u;
  a.pops = pops;
  const dim3 grid(blocks_for(g.S, 256)), block(256);
  dispatch_store_q(c, [&](auto st, auto q) {
    hipLaunchKernelGGL((k_read<decltype(st)::value, decltype(q)::value>), grid, block, 0, c->stream, a);
  });
  return hipGetLastError();
}

hipError_t launch_read_fields(lb_ctx* c, float* rho, float* u) { return launch_read(c, rho, u, nullptr); }

hipError_t launch_read_populations(lb_ctx* c, float* g) { return launch_read(c, nullptr, nullptr, g); }

hipError_t launch_write_populations(lb_ctx* c, const float* g) {
  const Geometry& geo = c->geo;
  WriteArgs a;
  a.f = c->popbuf[c->cur];
  a.plane = geo.plane;
  a.nx = geo.nx;
  a.ny = geo.ny;
  a.nz = geo.nz;
  a.S = (int)geo.S;
  a.pops = g;
  const dim3 grid(blocks_for(geo.S, 256)), block(256);
  dispatch_store_q(c, [&](auto st, auto q) {
    hipLaunchKernelGGL((k_write<decltype(st)::value, decltype(q)::value>), grid, block, 0, c->stream, a);
  });
  return hipGetLastError();
}

// ---- scratch of lb_invariants_noalloc ---------------------------------------------------------
// The per-workgroup partial sums of the FP64 reduction in a fixed array of the library's own
// device memory, one copy on every GPU the library runs on, held until the process ends (its
// size does not depend on the lattice: each reduction workgroup loops over sites).  In host
// code the name `scratch` is a host-side stand-in, not a device address: every host use goes
// through the address that setup_invariants_scratch() looks up once per device.
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t setup_invariants_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<double*>(p);
  return hipSuccess;
}

double* invariants_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

int invariants_blocks(const lb_ctx* c) {
  const int nb = blocks_for(c->geo.S, 256);
  return nb > kRedBlocks ? kRedBlocks : nb;
}

hipError_t launch_invariants(lb_ctx* c, double* partial, double* out) {
  const Geometry& g = c->geo;
  RedArgs a;
  a.f = c->popbuf[c->cur];
  a.plane = g.plane;
  a.S = (int)g.S;
  a.partial = partial;
  a.err = (uint32_t*)(c->ws + c->lay.err);
  const int nb = invariants_blocks(c);
  dispatch_store_q(c, [&](auto st, auto q) {
    hipLaunchKernelGGL((k_reduce_pops<decltype(st)::value, decltype(q)::value>), dim3(nb), dim3(256), 0,
                       c->stream, a);
  });
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  FinalArgs f;
  f.partial = a.partial;
  f.nblocks = nb;
  f.vel = (const float*)(c->ws + c->lay.vel);
  f.N = c->p.n_atoms;
  f.mass = c->p.mass;
  f.rest_mass = (double)c->p.rho0 * (double)g.S;
  f.out = out;
  f.err = a.err;
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, c->stream, f);
  return hipGetLastError();
}

}  // namespace lbmd
