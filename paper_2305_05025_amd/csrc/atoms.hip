// Atom-side kernels for gfx950: friction coupling to the lattice and the stand-in force
// field.
//
// Coupling (paper Section 2.2, friction-coupling paragraph): the fluid velocity at an atom
// is the linear interpolation over its eight nearest nodes, the atom feels
// F_c = gamma (U - v), and the fluid receives -F_c through the forcing term with the same
// eight trilinear weights.  The fluid velocity at a node is u_c = (j + F_ext/2)/rho of the
// pre-collision state (Eqs. 2-3); the atoms' own force is not included.
//
// Per step:
//   k_prep      clear the neighbour-list counts and the force-tile flags
//   k_bin_mark  one thread per atom: flag its 8 stencil nodes (plain byte stores) and their
//               64-site tiles, append the atom to the list of its stencil base node (lower
//               corner), and append a record of it to its neighbour-list cell
//   k_compact   lists of the occupied cells and of the flagged tiles
//   k_node_compact  list of the flagged nodes (within the flagged tiles)
//   k_node_u    u_c at every flagged node, one thread per node, pulled once per node (19 or
//               27 loads) rather than once per atom corner
//   k_couple    eight lanes per atom: weighted u_c of its node, xor-shuffle sum -> U,
//               F_c = gamma (U - v)
//   k_spread    every flagged node (one thread each) gathers -W F_c from the atoms listed at
//               the 8 base nodes
//               whose stencil covers it, summed in 2^-40 fixed point (order-independent) and
//               stored as a float; no atomics on the force
//   (lattice sweep: adds the spread force on flagged tiles and clears the per-step buffers)
//   k_cell_sort each occupied cell's records in atom-index order
//   k_forces_cells  tethers, bonds and the pair terms (Lennard-Jones, implicit-solvent
//               Coulomb) at X^n, one wavefront per occupied cell with the 27 neighbour
//               cells staged in LDS, FP32 sums in a fixed order
//   k_integrate symplectic Euler update
//
// Positions are kept as the caller's unwrapped anchors x0 plus a displacement d.  Stencil
// fractions and pair vectors are formed from small numbers only (fractions in [0, 1) and
// small integer offsets), so they keep full FP32 precision at any box size.
#include <climits>

#include "atoms_common.h"

namespace lbmd {
namespace {

// ------------------------------------------------------------------------------------------
struct PrepArgs {
  int* cell_count;
  long ncell;
  uint32_t* tile_flag;
  int ntiles;
  int* occ_count;
};

__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
  const long t = blockIdx.x * 256L + threadIdx.x;
  if (t < a.ncell) a.cell_count[t] = 0;
  if (t < a.ntiles) a.tile_flag[t] = 0u;
  if (t < 3) a.occ_count[t] = 0;
}

// ------------------------------------------------------------------------------------------
// Stream compaction of the occupied neighbour-list cells and of the flagged force tiles:
// one ballot and one counter atomic per wavefront.  The lists' order depends on scheduling;
// every consumer treats each entry independently, so results do not.
struct CompactArgs {
  const int* cell_count;
  long ncell;
  int* occ_cells;
  const uint32_t* tile_flag;
  int ntiles;
  int* occ_tiles;
  int* occ_count;
};

// block-wide compaction: one counter atomic per workgroup that has anything to append
__device__ __forceinline__ void compact_block(bool keep, int item, int* list, int* count) {
  __shared__ int wave_n[4];
  __shared__ int block_base;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const unsigned long long m = __ballot(keep);
  if (lane == 0) wave_n[wid] = __popcll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = wave_n[0] + wave_n[1] + wave_n[2] + wave_n[3];
    block_base = tot ? atomicAdd(count, tot) : 0;
  }
  __syncthreads();
  int off = block_base;
  for (int w = 0; w < wid; ++w) off += wave_n[w];
  if (keep) list[off + __popcll(m & ((1ull << lane) - 1ull))] = item;
}

// The flagged nodes inside the flagged tiles.  Each workgroup takes a contiguous range of the
// tile list and each of its wavefronts a contiguous quarter of that, so the list keeps the
// tiles' order within a workgroup (consecutive entries are neighbouring sites, which the node
// kernels' gathers rely on); the workgroup counts its flagged nodes, reserves room with a
// single counter atomic, then writes them in a second pass over the same tiles.  Tiles are
// visited four at a time with their loads issued together: this kernel runs beside the
// sweep, where every memory round trip is long.
struct NodeCompactArgs {
  int S;
  const int* occ_tiles;
  const uint8_t* node_flag;
  int* node_list;
  int* occ_count;    // [1] tiles (in), [2] nodes (out)
};

constexpr int kNodeBatch = 4;

// flags of this lane's site in tiles k .. k+3 of the list (0 past t1)
__device__ __forceinline__ void tile_flags(const NodeCompactArgs& a, int k, int t1, int lane,
                                           int (&s)[kNodeBatch], bool (&f)[kNodeBatch]) {
  int tile[kNodeBatch];
#pragma unroll
  for (int j = 0; j < kNodeBatch; ++j) tile[j] = k + j < t1 ? a.occ_tiles[k + j] : -1;
  uint8_t v[kNodeBatch];
#pragma unroll
  for (int j = 0; j < kNodeBatch; ++j) {
    s[j] = (tile[j] << kTileShift) + lane;
    v[j] = a.node_flag[tile[j] >= 0 && s[j] < a.S ? s[j] : 0];   // unconditional load
  }
#pragma unroll
  for (int j = 0; j < kNodeBatch; ++j) f[j] = tile[j] >= 0 && s[j] < a.S && v[j] != 0;
}

__global__ __launch_bounds__(256) void k_node_compact(NodeCompactArgs a) {
  __shared__ int wave_n[4];
  __shared__ int block_base;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int ntile = a.occ_count[1];
  const int chunk = (ntile + (int)gridDim.x - 1) / (int)gridDim.x;
  const int q = (chunk + 3) / 4;
  const int t0 = min((int)blockIdx.x * chunk + wid * q, ntile);
  const int t1 = min(min(t0 + q, (int)(blockIdx.x + 1) * chunk), ntile);
  int n = 0;
  for (int k = t0; k < t1; k += kNodeBatch) {
    int s[kNodeBatch];
    bool f[kNodeBatch];
    tile_flags(a, k, t1, lane, s, f);
#pragma unroll
    for (int j = 0; j < kNodeBatch; ++j) n += __popcll(__ballot(f[j]));
  }
  if (lane == 0) wave_n[wid] = n;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int tot = wave_n[0] + wave_n[1] + wave_n[2] + wave_n[3];
    block_base = tot ? atomicAdd(a.occ_count + 2, tot) : 0;
  }
  __syncthreads();
  int off = block_base;
  for (int w = 0; w < wid; ++w) off += wave_n[w];
  for (int k = t0; k < t1; k += kNodeBatch) {
    int s[kNodeBatch];
    bool f[kNodeBatch];
    tile_flags(a, k, t1, lane, s, f);
#pragma unroll
    for (int j = 0; j < kNodeBatch; ++j) {
      const unsigned long long m = __ballot(f[j]);
      if (f[j]) a.node_list[off + __popcll(m & ((1ull << lane) - 1ull))] = s[j];
      off += __popcll(m);
    }
  }
}

__global__ __launch_bounds__(256) void k_compact(CompactArgs a) {
  const long t = blockIdx.x * 256L + threadIdx.x;
  const long n_cell_blocks = (a.ncell + 255) / 256;
  if ((long)blockIdx.x < n_cell_blocks) {
    compact_block(t < a.ncell && a.cell_count[t] > 0, (int)t, a.occ_cells, a.occ_count);
  } else {
    const long u = t - n_cell_blocks * 256;
    compact_block(u < a.ntiles && a.tile_flag[u] != 0u, (int)u, a.occ_tiles, a.occ_count + 1);
  }
}

// ------------------------------------------------------------------------------------------
// Order each occupied cell's records by atom index (their slots came from atomics), so that
// the pair sums below run in a fixed order: one wavefront per occupied cell, lane = slot,
// rank by shuffles, then every lane writes its record to its rank.
struct SortArgs {
  const int* occ_cells;
  const int* occ_count;
  const int* cell_count;
  int4* cell_rec;
};

__global__ __launch_bounds__(256) void k_cell_sort(SortArgs a) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * 256 + threadIdx.x) >> 6, nwave = gridDim.x * 4;
  const int nocc = *a.occ_count;
  for (int k = wave; k < nocc; k += nwave) {
    const long cell = a.occ_cells[k];
    int n = a.cell_count[cell];
    n = n > kCellCap ? kCellCap : n;
    const bool mine = lane < n;
    const int4 rec = mine ? a.cell_rec[cell * kCellCap + lane] : make_int4(0, 0, 0, 0x7fffffff);
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += __shfl(rec.w, j, 64) < rec.w ? 1 : 0;
    if (mine) a.cell_rec[cell * kCellCap + rank] = rec;
  }
}

// ------------------------------------------------------------------------------------------
struct BinArgs {
  int N;
  AtomGeo g;
  const float* x0;
  const float* d;     // [2][N][3]: hi, lo
  uint32_t* tile_flag;
  uint8_t* node_flag;
  int* base_count;
  int* base_list;     // [plane][kBaseCap]
  float4* atom_frac;  // [N]: stencil fractions
  int* cell_count;
  int4* cell_rec;     // [ncell][kCellCap]: fixed-point position in the cell xyz, atom index
  uint32_t* err;
};

__global__ __launch_bounds__(256) void k_bin_mark(BinArgs a) {
  const int i = xcd_block() * 256 + threadIdx.x;
  if (i >= a.N) return;
  int i0[3];
  float fr[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    split(a.x0[3 * i + c], a.d[3 * i + c], a.d[3 * a.N + 3 * i + c], a.g.n[c], i0[c], fr[c]);
  const int x1 = i0[0] + 1 == a.g.n[0] ? 0 : i0[0] + 1;
  const int y1 = i0[1] + 1 == a.g.n[1] ? 0 : i0[1] + 1;
  const int z1 = i0[2] + 1 == a.g.n[2] ? 0 : i0[2] + 1;
  const int nx = a.g.n[0], nxy = a.g.n[0] * a.g.n[1];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int node = ((k & 1) ? x1 : i0[0]) + nx * ((k & 2) ? y1 : i0[1]) + nxy * ((k & 4) ? z1 : i0[2]);
    a.node_flag[node] = 1;
    a.tile_flag[node >> kTileShift] = 1u;
  }
  a.atom_frac[i] = make_float4(fr[0], fr[1], fr[2], 0.f);
  const int base = i0[0] + nx * i0[1] + nxy * i0[2];
  const int bslot = atomicAdd(a.base_count + base, 1);
  if (bslot < kBaseCap)
    a.base_list[(size_t)base * kBaseCap + bslot] = i;
  else
    atomicOr(a.err, kErrOverflow);
  if (a.g.nc[0] > 0) {
    int q[3], P[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      q[c] = cell_of(i0[c], fr[c], a.g.inv_cw[c], a.g.nc[c]);
      P[c] = cell_fixed(i0[c] - cell_origin(q[c], a.g.n[c], a.g.nc[c]), fr[c]);
    }
    const long cell = q[0] + (long)a.g.nc[0] * (q[1] + (long)a.g.nc[1] * q[2]);
    const int slot = atomicAdd(a.cell_count + cell, 1);
    if (slot < kCellCap)
      a.cell_rec[cell * kCellCap + slot] = make_int4(P[0], P[1], P[2], i);
    else
      atomicOr(a.err, kErrOverflow);
  }
}

// ------------------------------------------------------------------------------------------
// Binning of the fused coupled sweep.  One thread per atom: the atom joins the list of every
// brick that one of its 8 stencil nodes lies in (up to 8; a brick's list thus holds every atom
// whose interpolation or spread touches the brick), and a record of it joins its
// neighbour-list cell as in k_bin_mark.  List order comes from atomics; the hot-brick sweep
// treats every listed atom on its own and sums the spread in integers, so results do not
// depend on it.
struct BrickBinArgs {
  int N;
  AtomGeo g;
  int nb0, nb1;         // bricks along x and y
  const float* x0;
  const float* d;       // [2][N][3]: hi, lo
  int* brick_count;
  int* brick_list;      // [nbricks][kBrickCap]
  int* cell_count;
  int4* cell_rec;       // [ncell][kCellCap]
  uint32_t* err;
};

__global__ __launch_bounds__(256) void k_brick_bin(BrickBinArgs a) {
  const int i = xcd_block() * 256 + threadIdx.x;
  if (i >= a.N) return;   // (lanes that leave are inactive in the ballots below)
  int i0[3];
  float fr[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    split(a.x0[3 * i + c], a.d[3 * i + c], a.d[3 * a.N + 3 * i + c], a.g.n[c], i0[c], fr[c]);
  const int x1 = i0[0] + 1 == a.g.n[0] ? 0 : i0[0] + 1;
  const int y1 = i0[1] + 1 == a.g.n[1] ? 0 : i0[1] + 1;
  const int z1 = i0[2] + 1 == a.g.n[2] ? 0 : i0[2] + 1;
  const int bx[2] = {i0[0] >> kBrickShiftX, x1 >> kBrickShiftX};
  const int by[2] = {i0[1] >> kBrickShiftY, y1 >> kBrickShiftY};
  const int bz[2] = {i0[2] >> kBrickShiftZ, z1 >> kBrickShiftZ};
  // Neighbouring atoms (consecutive along a chain) mostly share bricks, so the lanes of a
  // wavefront that append to the same brick reserve their slots with one atomic between them.
  const unsigned long long below = (1ull << (threadIdx.x & 63)) - 1ull;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
    // each distinct brick of this atom once
    const bool dup = (dx && bx[1] == bx[0]) || (dy && by[1] == by[0]) || (dz && bz[1] == bz[0]);
    long b = dup ? -1 : bx[dx] + (long)a.nb0 * (by[dy] + (long)a.nb1 * bz[dz]);
    while (__ballot(b >= 0) != 0ull) {
      const unsigned long long act = __ballot(b >= 0);
      const int leader = __ffsll((long long)act) - 1;
      const long bl = __shfl(b, leader, 64);
      const unsigned long long same = __ballot(b == bl);
      int base = 0;
      if ((int)(threadIdx.x & 63) == leader) base = atomicAdd(a.brick_count + bl, __popcll(same));
      base = __shfl(base, leader, 64);
      if (b == bl) {
        const int slot = base + __popcll(same & below);
        if (slot < kBrickCap)
          a.brick_list[bl * kBrickCap + slot] = i;
        else
          atomicOr(a.err, kErrOverflow);
        b = -1;
      }
    }
  }
  if (a.g.nc[0] > 0) {
    int q[3], P[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      q[c] = cell_of(i0[c], fr[c], a.g.inv_cw[c], a.g.nc[c]);
      P[c] = cell_fixed(i0[c] - cell_origin(q[c], a.g.n[c], a.g.nc[c]), fr[c]);
    }
    const long cell = q[0] + (long)a.g.nc[0] * (q[1] + (long)a.g.nc[1] * q[2]);
    const int slot = atomicAdd(a.cell_count + cell, 1);
    if (slot < kCellCap)
      a.cell_rec[cell * kCellCap + slot] = make_int4(P[0], P[1], P[2], i);
    else
      atomicOr(a.err, kErrOverflow);
  }
}

// ------------------------------------------------------------------------------------------
struct NodeArgs {
  const void* f;
  long plane;
  int nx, ny, nz, S;
  float rho0;
  int bf_kind;
  const float* fext_tab;
  const float* fext_field;
  const int* node_list;
  const int* node_count;
  float* uc;   // [3][plane]
  FastDiv dnx, dny;
  int narrow;  // planes take 32-bit byte offsets
};

// one thread per flagged node (persistent over the node list)
template <int ST, int Q>
__global__ __launch_bounds__(256) void k_node_u(NodeArgs a) {
  using T = typename Store<ST>::T;
  const int n = *a.node_count;
  for (int k = blockIdx.x * 256 + threadIdx.x; k < n; k += gridDim.x * 256) {
    const int s = a.node_list[k];
    int x, y, z;
    site_xyz(s, a.nx, a.ny, a.dnx, a.dny, x, y, z);
    float g[Q];
    gather<ST, Q>(reinterpret_cast<const T*>(a.f), a.plane, x, y, z, a.nx, a.ny, a.nz,
                  a.narrow != 0, g);
    float drho, jx, jy, jz, Fx, Fy, Fz;
    moments<Q>(g, drho, jx, jy, jz);
    external_force(a.bf_kind, a.fext_tab, a.fext_field, a.plane, s, y, Fx, Fy, Fz);
    const float inv = 1.0f / (a.rho0 + drho);
    a.uc[s] = (jx + 0.5f * Fx) * inv;
    a.uc[a.plane + s] = (jy + 0.5f * Fy) * inv;
    a.uc[2 * a.plane + s] = (jz + 0.5f * Fz) * inv;
  }
}

// ------------------------------------------------------------------------------------------
struct CoupleArgs {
  int N;
  int n[3];
  long plane;
  float gamma;
  const float* x0;
  const float* d;         // [2][N][3]: hi, lo
  const float* v;         // [2][N][3]: hi, lo
  const float* uc;
  float* fc;              // out: friction force on each atom
  float* U;               // out, optional: interpolated fluid velocity at each atom
};

__global__ __launch_bounds__(256) void k_couple(CoupleArgs a) {
  const int tid = xcd_block() * 256 + threadIdx.x;
  const int atom = tid >> 3;
  const int k = tid & 7;
  const bool valid = atom < a.N;
  const int at = valid ? atom : a.N - 1;
  int i0[3];
  float fr[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
    split(a.x0[3 * at + c], a.d[3 * at + c], a.d[3 * a.N + 3 * at + c], a.n[c], i0[c], fr[c]);
  const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
  const int x = dx ? (i0[0] + 1 == a.n[0] ? 0 : i0[0] + 1) : i0[0];
  const int y = dy ? (i0[1] + 1 == a.n[1] ? 0 : i0[1] + 1) : i0[1];
  const int z = dz ? (i0[2] + 1 == a.n[2] ? 0 : i0[2] + 1) : i0[2];
  const float w = (dx ? fr[0] : 1.0f - fr[0]) * (dy ? fr[1] : 1.0f - fr[1]) *
                  (dz ? fr[2] : 1.0f - fr[2]);
  const int node = x + a.n[0] * (y + a.n[1] * z);
  float Ux = w * a.uc[node];
  float Uy = w * a.uc[a.plane + node];
  float Uz = w * a.uc[2 * a.plane + node];
  // sum over the 8 lanes of this atom (lanes 8a..8a+7 of the wavefront)
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) {
    Ux += __shfl_xor(Ux, o, 64);
    Uy += __shfl_xor(Uy, o, 64);
    Uz += __shfl_xor(Uz, o, 64);
  }
  if (!valid || k != 0) return;
  if (a.U) {
    a.U[3 * atom] = Ux;
    a.U[3 * atom + 1] = Uy;
    a.U[3 * atom + 2] = Uz;
  }
  const float* vlo = a.v + 3 * a.N;
  a.fc[3 * atom] = a.gamma * ((Ux - a.v[3 * atom]) - vlo[3 * atom]);
  a.fc[3 * atom + 1] = a.gamma * ((Uy - a.v[3 * atom + 1]) - vlo[3 * atom + 1]);
  a.fc[3 * atom + 2] = a.gamma * ((Uz - a.v[3 * atom + 2]) - vlo[3 * atom + 2]);
}

// ------------------------------------------------------------------------------------------
struct SpreadArgs {
  int S;
  int n[3];
  long plane;
  const int* node_list;
  const int* node_count;
  uint8_t* node_flag;        // cleared here
  const int* base_count;
  const int* base_list;
  const float4* atom_frac;
  const float* fc;
  float* fcoup;              // [3][plane]
};

// The transpose of the interpolation: node x is corner delta of every atom whose base node
// is x - delta; its share of that atom's -F_c is the same trilinear weight.  One thread per
// flagged node (persistent over the node list).
__global__ __launch_bounds__(256) void k_spread(SpreadArgs a) {
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const int n = *a.node_count;
  for (int kn = blockIdx.x * 256 + threadIdx.x; kn < n; kn += gridDim.x * 256) {
    const int s = a.node_list[kn];
    const int x = s % nx;
    const int t = s / nx;
    const int y = t % ny;
    const int z = t / ny;
    // the 8 candidate base nodes; their counts and first two list entries are loaded up front
    // (independent loads; every site owns kBaseCap list slots, and an entry is used only
    // below its count)
    int base[8], nb[8], e0[8], e1[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
      const int bx = dx ? (x == 0 ? nx - 1 : x - 1) : x;
      const int by = dy ? (y == 0 ? ny - 1 : y - 1) : y;
      const int bz = dz ? (z == 0 ? nz - 1 : z - 1) : z;
      base[k] = bx + nx * (by + ny * bz);
      nb[k] = a.base_count[base[k]];
      e0[k] = a.base_list[(size_t)base[k] * kBaseCap];
      e1[k] = a.base_list[(size_t)base[k] * kBaseCap + 1];
    }
    long long Sx = 0, Sy = 0, Sz = 0;
    // entry q of every corner in one round: the round's loads are all in flight before the
    // first is used (a corner without entry q reads atom 0's values and skips them).  The
    // fixed-point sum does not depend on the order of its terms.
    auto add_round = [&](const int (&e)[8], int q) {
      float4 fr[8];
      float fx[8], fy[8], fz[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int at = nb[k] > q ? e[k] : 0;
        fr[k] = a.atom_frac[at];
        fx[k] = a.fc[3 * at];
        fy[k] = a.fc[3 * at + 1];
        fz[k] = a.fc[3 * at + 2];
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (nb[k] <= q) continue;
        const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
        const float w = (dx ? fr[k].x : 1.0f - fr[k].x) * (dy ? fr[k].y : 1.0f - fr[k].y) *
                        (dz ? fr[k].z : 1.0f - fr[k].z);
        Sx += to_fixed(-w * fx[k], kFixScale);
        Sy += to_fixed(-w * fy[k], kFixScale);
        Sz += to_fixed(-w * fz[k], kFixScale);
      }
    };
    add_round(e0, 0);
    add_round(e1, 1);
    // entries 2 .. count-1 (base nodes holding more than two atoms)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int dx = k & 1, dy = (k >> 1) & 1, dz = (k >> 2) & 1;
      const int n = nb[k] > kBaseCap ? kBaseCap : nb[k];
      for (int q = 2; q < n; ++q) {
        const int at = a.base_list[(size_t)base[k] * kBaseCap + q];
        const float4 fr = a.atom_frac[at];
        const float w = (dx ? fr.x : 1.0f - fr.x) * (dy ? fr.y : 1.0f - fr.y) * (dz ? fr.z : 1.0f - fr.z);
        Sx += to_fixed(-w * a.fc[3 * at], kFixScale);
        Sy += to_fixed(-w * a.fc[3 * at + 1], kFixScale);
        Sz += to_fixed(-w * a.fc[3 * at + 2], kFixScale);
      }
    }
    a.fcoup[s] = (float)Sx * kFixInv;
    a.fcoup[a.plane + s] = (float)Sy * kFixInv;
    a.fcoup[2 * a.plane + s] = (float)Sz * kFixInv;
    a.node_flag[s] = 0;
  }
}

// ------------------------------------------------------------------------------------------
struct ForceArgs {
  int N;
  AtomGeo g;
  long ncell;
  float L[3], invL[3];
  const float* x0;
  const float* d;       // X^n - x0: [2][N][3], hi then lo
  float* ff;            // out: stand-in force field at X^n
  float k_tether;
  const int* bond_off;
  const int* bond_nbr;
  float k_bond, r0_bond;
  float lj_eps24, lj_sigma2, lj_rc2;
  int lj_exclude_bonded;
  float coul2;            // 2 k_C (0: no Coulomb term)
  const float* charge;
  const int* cell_count;
  const int4* cell_rec;
  const int* occ_cells;
  const int* occ_count;   // [1]: number of occupied cells
  uint32_t* err;
  // Hessian-vector product (adjoint) only: direction per atom, and lx_out = lx_in + H lf
  const float4* lf;
  const float* lx_in;
  float* lx_out;
};

// Tethers and bonds of atom i added to its pair-term part.  Forward: the total stand-in
// force field at X^n is stored for the integration.  Adjoint (kAdj): the same terms of the
// force Jacobian applied to the direction lf (the Jacobian is symmetric), added to lx_in.
// For a pair term f(r) = g(|r|^2) r with r = X_i - X_j, the Jacobian block is
// J = g I + 2 g' r r^T, and atom i receives J (lf_i - lf_j).
template <bool kAdj>
__device__ __forceinline__ void add_bond(const ForceArgs& a, float rx, float ry, float rz,
                                         float4 li, float4 lj, float& Fx, float& Fy, float& Fz) {
  const float rl = sqrtf(rx * rx + ry * ry + rz * rz);
  const float f = -a.k_bond * (rl - a.r0_bond) / rl;
  if constexpr (kAdj) {
    // g = -k (1 - r0/|r|), 2 g' = -k r0 / |r|^3
    const float ex = li.x - lj.x, ey = li.y - lj.y, ez = li.z - lj.z;
    const float t = -a.k_bond * a.r0_bond / (rl * rl * rl) * (rx * ex + ry * ey + rz * ez);
    Fx += f * ex + t * rx;
    Fy += f * ey + t * ry;
    Fz += f * ez + t * rz;
  } else {
    Fx += f * rx;
    Fy += f * ry;
    Fz += f * rz;
  }
}

constexpr int kBondPre = 4;   // bond partners whose positions are loaded together, up front

template <bool kAdj>
__device__ __forceinline__ void bonded_and_store(const ForceArgs& a, int i, float Fx, float Fy,
                                                 float Fz) {
  const float xi = a.x0[3 * i], yi = a.x0[3 * i + 1], zi = a.x0[3 * i + 2];
  // displacement differences: hi parts of nearby atoms subtract exactly, then the lo parts
  const float* dlo = a.d + 3 * a.N;
  const float dxi = a.d[3 * i], dyi = a.d[3 * i + 1], dzi = a.d[3 * i + 2];
  const float lxi = dlo[3 * i], lyi = dlo[3 * i + 1], lzi = dlo[3 * i + 2];
  const int b0 = a.bond_off[i], b1 = a.bond_off[i + 1];
  // the first kBondPre partners (atom i itself stands in for a missing one): all loads are
  // in flight before the first is used
  int pj[kBondPre];
#pragma unroll
  for (int k = 0; k < kBondPre; ++k) pj[k] = b0 + k < b1 ? a.bond_nbr[b0 + k] : i;
  float xj[kBondPre][3], dj[kBondPre][3], lj_[kBondPre][3];
  float4 lj[kBondPre];
#pragma unroll
  for (int k = 0; k < kBondPre; ++k) {
    const int j = pj[k];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      xj[k][d] = a.x0[3 * j + d];
      dj[k][d] = a.d[3 * j + d];
      lj_[k][d] = dlo[3 * j + d];
    }
    lj[k] = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (kAdj) lj[k] = a.lf[j];
  }
  float4 li = make_float4(0.f, 0.f, 0.f, 0.f);
  if constexpr (kAdj) {
    li = a.lf[i];
    Fx -= a.k_tether * li.x;
    Fy -= a.k_tether * li.y;
    Fz -= a.k_tether * li.z;
  } else {
    Fx -= a.k_tether * dxi;
    Fy -= a.k_tether * dyi;
    Fz -= a.k_tether * dzi;
  }
  // bonds in list order
#pragma unroll
  for (int k = 0; k < kBondPre; ++k) {
    if (b0 + k >= b1) break;
    add_bond<kAdj>(a, min_image((xi - xj[k][0]) + ((dxi - dj[k][0]) + (lxi - lj_[k][0])), a.L[0], a.invL[0]),
                   min_image((yi - xj[k][1]) + ((dyi - dj[k][1]) + (lyi - lj_[k][1])), a.L[1], a.invL[1]),
                   min_image((zi - xj[k][2]) + ((dzi - dj[k][2]) + (lzi - lj_[k][2])), a.L[2], a.invL[2]),
                   li, lj[k], Fx, Fy, Fz);
  }
  for (int b = b0 + kBondPre; b < b1; ++b) {
    const int j = a.bond_nbr[b];
    float4 l = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (kAdj) l = a.lf[j];
    add_bond<kAdj>(a, min_image((xi - a.x0[3 * j]) + ((dxi - a.d[3 * j]) + (lxi - dlo[3 * j])), a.L[0], a.invL[0]),
                   min_image((yi - a.x0[3 * j + 1]) + ((dyi - a.d[3 * j + 1]) + (lyi - dlo[3 * j + 1])), a.L[1], a.invL[1]),
                   min_image((zi - a.x0[3 * j + 2]) + ((dzi - a.d[3 * j + 2]) + (lzi - dlo[3 * j + 2])), a.L[2], a.invL[2]),
                   li, l, Fx, Fy, Fz);
  }
  if constexpr (kAdj) {
    a.lx_out[3 * i] = a.lx_in[3 * i] + Fx;
    a.lx_out[3 * i + 1] = a.lx_in[3 * i + 1] + Fy;
    a.lx_out[3 * i + 2] = a.lx_in[3 * i + 2] + Fz;
  } else {
    a.ff[3 * i] = Fx;
    a.ff[3 * i + 1] = Fy;
    a.ff[3 * i + 2] = Fz;
  }
}

// Pair terms (Lennard-Jones, implicit-solvent Coulomb; each cut off at r_c and shifted so
// that its force vanishes there), cell-centric, staged in LDS.  A wavefront takes one occupied cell at a time
// (persistent over the occupied-cell list):
//   1. lanes 0..26 find the 27 neighbour cells (with the periodic shift of each) and their
//      counts; a wave scan gives each cell's offset in the concatenation of their records;
//   2. the records of as many whole cells as fit are read (further rounds take the rest),
//      shifted into the home cell's frame, and those within the cut-off of the home atoms'
//      bounding box are copied into LDS in their original order.  Lanes cover record slots,
//      not cells: a lane finds the cell of each of its slots by a lower-bound search over
//      the scan, so every load of a round is in flight before the first is used.  Charges
//      (with the Coulomb term) and the adjoint's directions are staged beside the records;
//   3. the 64 lanes are split into G = floor(64 / nh) groups of nh lanes, nh the number of
//      home atoms (lane = group * nh + home slot; the remaining lanes idle); group g takes
//      staged records g, g + G, ...; all lanes of a group read the same LDS record (a
//      broadcast).  Pairs beyond the cut-off, the atom itself and excluded bonded partners
//      contribute an exact zero (a select, so the loop has no branch).
// The box test only drops records that no home atom can reach (it keeps a 0.1% margin over
// FP32 rounding); every kept pair passes the same cut-off test as before, so the result
// does not depend on it.  Each lane sums in FP32 in a fixed order (records in cell order,
// atom-index order inside a cell); the group partials meet in LDS and group 0 adds them in
// ascending group order, then adds tethers and bonds and stores.  Pair vectors come from
// exact fixed-point differences.  Each atom sits in exactly one cell slot, so every atom is
// written once.
constexpr int kStage = 320;   // records read per staging round (27 cells of ~9 atoms: ~240)
constexpr int kStageRounds = kStage / 64;
constexpr int kStagePad = kStage + 64;   // room for the pair loop's read-ahead past the end

// kCoul: the implicit-solvent Coulomb term is on (coul2 != 0)
template <bool kAdj, bool kCoul>
__global__ __launch_bounds__(256) void k_forces_cells(ForceArgs a) {
  __shared__ int4 stage_all[4][kStagePad];
  __shared__ float stage_q_all[kCoul ? 4 : 1][kCoul ? kStagePad : 1];
  __shared__ float4 stage_l_all[kAdj ? 4 : 1][kAdj ? kStagePad : 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int4* stage = stage_all[wid];
  float* stage_q = stage_q_all[kCoul ? wid : 0];
  float4* stage_l = stage_l_all[kAdj ? wid : 0];
  constexpr bool coul = kCoul;
  const unsigned long long below = (1ull << lane) - 1ull;
  const float keep_r2 = a.lj_rc2 * 1.001f;
  // The forward instance works in fixed-point units (2^-24 lattice units): pair vectors are
  // the converted integer differences, and the constants carry the powers of two instead
  // (exact, so the arithmetic is that of lattice units).  The adjoint keeps lattice units.
  constexpr float kU = kAdj ? kCellFixInv : 1.0f;                  // fixed-point unit -> length
  constexpr float kU2 = kAdj ? 1.0f : 281474976710656.0f;          // 2^48: r^2 in units^2
  const float rc2_u = a.lj_rc2 * kU2, sig2_u = a.lj_sigma2 * kU2;
  const float eps24_u = a.lj_eps24 * (kAdj ? 1.0f : 16777216.0f);  // 2^24
  const float coul2_u = a.coul2 * (kAdj ? 1.0f : 4722366482869645213696.0f);   // 2^72
  // Each pair term is shifted by its value at the cut-off, g(s) = g0(s) - g0(r_c^2), so the
  // force falls continuously to zero at r_c (a pair whose distance rounds to either side of
  // r_c then changes the force by a rounding-sized amount, not by a jump); the Jacobian term
  // 2 g'(s) is that of g0.  Evaluated in the units above.
  const float sr6c = (sig2_u / rc2_u) * (sig2_u / rc2_u) * (sig2_u / rc2_u);
  const float lj_shift_u = eps24_u * (2.0f * sr6c * sr6c - sr6c) / rc2_u;
  const float inv_rc4_u = 1.0f / (rc2_u * rc2_u);
  const int nc0 = a.g.nc[0], nc1 = a.g.nc[1], nc2 = a.g.nc[2];
  // XCD x takes the x-th contiguous eighth of the occupied-cell list (the list runs in cell
  // order, so neighbouring cells are near each other in it), interleaved over its own
  // waves: the 27-cell neighbourhoods it stages then overlap in that XCD's L2.  The grid is
  // a multiple of 8 workgroups.
  const int nocc = *a.occ_count;
  const int chunk = (nocc + 7) >> 3;
  const int k0 = (int)(blockIdx.x & 7u) * chunk, k1 = min(k0 + chunk, nocc);
  const int lwave = (int)(blockIdx.x >> 3) * 4 + wid, nlwave = (int)(gridDim.x >> 3) * 4;
  for (int k = k0 + lwave; k < k1; k += nlwave) {
    const int cell = a.occ_cells[k];
    int nh = a.cell_count[cell];
    nh = nh > kCellCap ? kCellCap : nh;
    nh = nh < 1 ? 1 : nh;   // listed cells are occupied; kept for the division below
    const int ngrp = 64 / nh;
    const int grp = lane / nh, hl = lane - grp * nh;
    const int cxy = cell / nc0;
    const int q[3] = {cell - cxy * nc0, cxy % nc1, cxy / nc1};
    // this lane's home atom (lanes 0..nh-1 hold the nh home atoms)
    const bool hv = grp < ngrp;
    const int4 me = a.cell_rec[(long)cell * kCellCap + (hv ? hl : 0)];
    const int i = me.w;
    const int b0 = a.bond_off[i], b1 = a.bond_off[i + 1];
    int pb[4] = {-1, -1, -1, -1};
    if (a.lj_exclude_bonded) {
      const int deg = b1 - b0;
      if (deg > 0) pb[0] = a.bond_nbr[b0];
      if (deg > 1) pb[1] = a.bond_nbr[b0 + 1];
      if (deg > 2) pb[2] = a.bond_nbr[b0 + 2];
      if (deg > 3) pb[3] = a.bond_nbr[b0 + 3];
    }
    // atoms with more than four bonded partners check the rest of their list in the pair
    // loop (a branch taken by the whole wavefront, rare)
    const bool many = __ballot(hv && a.lj_exclude_bonded && b1 - b0 > 4) != 0ull;
    float4 lfi = make_float4(0.f, 0.f, 0.f, 0.f);
    if constexpr (kAdj) lfi = a.lf[i];
    float qi = 0.f;
    if constexpr (coul) qi = a.charge[i];
    // bounding box of the home atoms (fixed point, home frame)
    int lo[3] = {lane < nh ? me.x : INT_MAX, lane < nh ? me.y : INT_MAX, lane < nh ? me.z : INT_MAX};
    int hi[3] = {lane < nh ? me.x : INT_MIN, lane < nh ? me.y : INT_MIN, lane < nh ? me.z : INT_MIN};
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = min(lo[d], __shfl_xor(lo[d], o, 64));
        hi[d] = max(hi[d], __shfl_xor(hi[d], o, 64));
      }
    float Fx = 0.f, Fy = 0.f, Fz = 0.f;
    // neighbour cells: lane l < 27 holds cell l of the 3x3x3 block
    int nbc = 0;
    int nbn = 0, shx = 0, shy = 0, shz = 0;
    if (lane < 27) {
      int cx, cy, cz;
      nbr_cell(q[0], lane % 3 - 1, a.g.n[0], nc0, cx, shx);
      nbr_cell(q[1], (lane / 3) % 3 - 1, a.g.n[1], nc1, cy, shy);
      nbr_cell(q[2], lane / 9 - 1, a.g.n[2], nc2, cz, shz);
      nbc = cx + nc0 * (cy + nc1 * cz);
      nbn = a.cell_count[nbc];
      nbn = nbn > kCellCap ? kCellCap : nbn;
    }
    int pre = nbn;   // inclusive scan over lanes 0..31 (only lanes 0..26 are read)
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      const int t = __shfl_up(pre, o, 64);
      if (lane >= o) pre += t;
    }
    const int pex = pre - nbn;   // first record of cell `lane` in the concatenation
    for (int kc = 0; kc < 27;) {
      const int base = __shfl(pex, kc, 64);
      // cells kc .. kend-1 fit (each cell holds at most kCellCap <= kStage records, so at
      // least one does); the cells that fit form a prefix of 0..26
      const int kend = __popcll(__ballot(lane < 27 && pre - base <= kStage));
      const int ntot = __shfl(pre, kend - 1, 64) - base;
      int4 rec[kStageRounds];
      int rc[kStageRounds];
#pragma unroll
      for (int r = 0; r < kStageRounds; ++r) {
        const int t = r * 64 + lane, gt = base + t;
        // lower bound: c = number of cells whose records all precede gt
        int c = 0;
#pragma unroll
        for (int step = 16; step >= 1; step >>= 1) {
          const int probe = c + step - 1;
          const int pv = __shfl(pre, probe < 26 ? probe : 26, 64);
          if (probe < 27 && pv <= gt) c += step;
        }
        c = c < 26 ? c : 26;
        const int j = gt - __shfl(pex, c, 64);
        const int cc = __shfl(nbc, c, 64);
        rc[r] = c;
        // slots past the end read the home cell's first record (valid, unused), so the
        // loads carry no branch
        rec[r] = a.cell_rec[t < ntot ? (long)cc * kCellCap + j : (long)cell * kCellCap];
      }
      int nkeep = 0, kpos[kStageRounds];
#pragma unroll
      for (int r = 0; r < kStageRounds; ++r) {
        const int c = rc[r];
        // neighbour position in the home cell's frame (fixed point)
        const int4 v = make_int4(rec[r].x - (__shfl(shx, c, 64) << 24),
                                 rec[r].y - (__shfl(shy, c, 64) << 24),
                                 rec[r].z - (__shfl(shz, c, 64) << 24), rec[r].w);
        const float ex = (float)max(max(lo[0] - v.x, v.x - hi[0]), 0) * kCellFixInv;
        const float ey = (float)max(max(lo[1] - v.y, v.y - hi[1]), 0) * kCellFixInv;
        const float ez = (float)max(max(lo[2] - v.z, v.z - hi[2]), 0) * kCellFixInv;
        const bool keep = r * 64 + lane < ntot && ex * ex + ey * ey + ez * ez < keep_r2;
        const unsigned long long m = __ballot(keep);
        kpos[r] = keep ? nkeep + __popcll(m & below) : -1;
        if (keep) stage[kpos[r]] = v;
        nkeep += __popcll(m);
      }
      // per-atom values of the staged records
      if constexpr (coul) {
        float qv[kStageRounds];
#pragma unroll
        for (int r = 0; r < kStageRounds; ++r) qv[r] = a.charge[rec[r].w];
#pragma unroll
        for (int r = 0; r < kStageRounds; ++r)
          if (kpos[r] >= 0) stage_q[kpos[r]] = qv[r];
      }
      if constexpr (kAdj) {
        float4 lv[kStageRounds];
#pragma unroll
        for (int r = 0; r < kStageRounds; ++r) lv[r] = a.lf[rec[r].w];
#pragma unroll
        for (int r = 0; r < kStageRounds; ++r)
          if (kpos[r] >= 0) stage_l[kpos[r]] = lv[r];
      }
      wave_lds_sync();
      if (hv) {
        // each record is read from LDS one iteration ahead of its use (reads past nkeep
        // stay inside the padded stage and are not used)
        int4 r_next = stage[grp];
        float q_next = 0.f;
        if constexpr (coul) q_next = stage_q[grp];
        float4 l_next = make_float4(0.f, 0.f, 0.f, 0.f);
        if constexpr (kAdj) l_next = stage_l[grp];
#pragma unroll 2
        for (int c = grp; c < nkeep; c += ngrp) {
          const int4 r4 = r_next;
          const float qj = q_next;
          const float4 lj = l_next;
          r_next = stage[c + ngrp];
          if constexpr (coul) q_next = stage_q[c + ngrp];
          if constexpr (kAdj) l_next = stage_l[c + ngrp];
          // pair vector X_i - X_j: exact integer difference, one rounding
          const float rx = (float)(me.x - r4.x) * kU;
          const float ry = (float)(me.y - r4.y) * kU;
          const float rz = (float)(me.z - r4.z) * kU;
          const float r2 = rx * rx + ry * ry + rz * rz;
          const int j = r4.w;
          // excluded bonded partners (pb holds -1 where there is none)
          bool bonded = j == pb[0] || j == pb[1] || j == pb[2] || j == pb[3];
          if (many)
            for (int bb = b0 + 4; bb < b1; ++bb) bonded = bonded || (a.bond_nbr[bb] == j);
          const bool use = r2 < rc2_u && j != i && !bonded;
          const float inv2 = __builtin_amdgcn_rcpf(r2);
          const float sr2 = sig2_u * inv2;
          const float sr6 = sr2 * sr2 * sr2;
          // force on i = g(s) r with s = r^2; LJ: g = 24 eps (2 sigma^12 s^-7 - sigma^6 s^-4)
          // (forward: g 2^-24, which turns the fixed-point r into lattice units)
          float f = eps24_u * (2.0f * sr6 * sr6 - sr6) * inv2 - lj_shift_u;
          // the Jacobian uses 2 g'(s)
          float gp2 = 0.f;
          if constexpr (kAdj) gp2 = 2.0f * a.lj_eps24 * (4.0f * sr6 - 14.0f * sr6 * sr6) * inv2 * inv2;
          if constexpr (coul) {
            // implicit-solvent Coulomb: g = 2 k_C q_i q_j s^-2, 2 g' = -4 g / s
            const float cq = coul2_u * qi * qj;
            const float gc = cq * inv2 * inv2;
            f += gc - cq * inv_rc4_u;
            if constexpr (kAdj) gp2 -= 4.0f * gc * inv2;
          }
          f = use ? f : 0.f;
          if constexpr (kAdj) {
            gp2 = use ? gp2 : 0.f;
            const float ex = lfi.x - lj.x, ey = lfi.y - lj.y, ez = lfi.z - lj.z;
            const float t = gp2 * (rx * ex + ry * ey + rz * ez);
            Fx += f * ex + t * rx;
            Fy += f * ey + t * ry;
            Fz += f * ez + t * rz;
          } else {
            Fx += f * rx;
            Fy += f * ry;
            Fz += f * rz;
          }
        }
      }
      wave_lds_sync();
      kc = kend;
    }
    // group partials, through this wavefront's stage: group 0 adds groups 1 .. G-1 in order
    float* part = reinterpret_cast<float*>(stage);
    if (ngrp > 1) {
      part[lane] = Fx;
      part[64 + lane] = Fy;
      part[128 + lane] = Fz;
      wave_lds_sync();
      if (grp == 0)
        for (int g = 1; g < ngrp; ++g) {
          Fx += part[g * nh + hl];
          Fy += part[64 + g * nh + hl];
          Fz += part[128 + g * nh + hl];
        }
      wave_lds_sync();
    }
    if (hv && grp == 0) bonded_and_store<kAdj>(a, i, Fx, Fy, Fz);
  }
}

// Without Lennard-Jones: one thread per atom, tethers + bonds.
template <bool kAdj>
__global__ __launch_bounds__(256) void k_bonded_forces(ForceArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.N) return;
  bonded_and_store<kAdj>(a, i, 0.f, 0.f, 0.f);
}

// Symplectic Euler with the force field at X^n and the friction of this step:
// v^{n+1} = v^n + (F_ff + F_c)/m, X^{n+1} = X^n + v^{n+1}: the velocity increment is
// rounded once, then added to the float-float velocity, which is added to the float-float
// displacement, both exactly.
struct IntegrateArgs {
  int N;
  float inv_mass;
  const float* ff;
  const float* fc;
  const float* d;       // [2][N][3] hi, lo
  float* d_next;        // [2][N][3]
  float* v;             // [2][N][3]
  uint32_t* err;
};

__global__ __launch_bounds__(256) void k_integrate(IntegrateArgs a) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= a.N) return;
  const int lo = 3 * a.N;
  bool finite = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int k = 3 * t + c;
    float vh = a.v[k], vl = a.v[lo + k];
    ff_add(vh, vl, (a.ff[k] + a.fc[k]) * a.inv_mass, 0.0f);
    finite = finite && __builtin_isfinite(vh);
    float dh = a.d[k], dl = a.d[lo + k];
    ff_add(dh, dl, vh, vl);
    a.v[k] = vh;
    a.v[lo + k] = vl;
    a.d_next[k] = dh;
    a.d_next[lo + k] = dl;
  }
  if (!finite) atomicOr(a.err, kErrNonFinite);
}

// unwrapped positions x0 + d and velocities, each rounded once from its exact sum
__global__ __launch_bounds__(256) void k_read_atoms(int N, const float* x0, const float* d,
                                                    const float* v, float* xo, float* vo) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= 3 * N) return;
  if (xo) {
    float s, e;
    two_sum(x0[t], d[t], s, e);
    xo[t] = s + (e + d[3 * N + t]);
  }
  if (vo) vo[t] = v[t] + v[3 * N + t];
}

}  // namespace

hipError_t launch_prep(lb_ctx* c) {
  PrepArgs a;
  a.cell_count = (int*)(c->bin + c->lay.cell_count);
  a.ncell = c->geo.ncell;
  a.tile_flag = (uint32_t*)(c->bin + c->lay.tile_flag[c->step & 1]);
  a.ntiles = c->geo.ntiles;
  a.occ_count = (int*)(c->bin + c->lay.occ_count[c->step & 1]);
  const long n = a.ncell > a.ntiles ? a.ncell : a.ntiles;
  hipLaunchKernelGGL(k_prep, dim3(blocks(n, 256)), dim3(256), 0, c->astream, a);
  return hipGetLastError();
}

hipError_t launch_compact(lb_ctx* c) {
  CompactArgs a;
  a.cell_count = (const int*)(c->bin + c->lay.cell_count);
  a.ncell = c->geo.ncell;
  a.occ_cells = (int*)(c->bin + c->lay.occ_cells);
  a.tile_flag = (const uint32_t*)(c->bin + c->lay.tile_flag[c->step & 1]);
  a.ntiles = c->geo.ntiles;
  a.occ_tiles = (int*)(c->bin + c->lay.occ_tiles[c->step & 1]);
  a.occ_count = (int*)(c->bin + c->lay.occ_count[c->step & 1]);
  const long nb = (a.ncell + 255) / 256 + (a.ntiles + 255) / 256;
  hipLaunchKernelGGL(k_compact, dim3((unsigned)nb), dim3(256), 0, c->astream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  NodeCompactArgs b;
  b.S = (int)c->geo.S;
  b.occ_tiles = a.occ_tiles;
  b.node_flag = (const uint8_t*)(c->ws + c->lay.node_flag);
  b.node_list = (int*)(c->bin + c->lay.node_list[c->step & 1]);
  b.occ_count = a.occ_count;
  hipLaunchKernelGGL(k_node_compact, dim3(1024), dim3(256), 0, c->astream, b);
  return hipGetLastError();
}

// clear the counts, bin, then list the occupied cells and the hot bricks (whose count is kept
// where the old path keeps its flagged-tile count, occ_count[1])
hipError_t launch_brick_binning(lb_ctx* c) {
  const int par = (int)(c->step & 1);
  PrepArgs p;
  p.cell_count = (int*)(c->bin + c->lay.cell_count);
  p.ncell = c->geo.ncell;
  p.tile_flag = (uint32_t*)(c->ws + c->lay.brick_count[par]);
  p.ntiles = (int)c->geo.nbricks;
  p.occ_count = (int*)(c->bin + c->lay.occ_count[par]);
  const long n = p.ncell > p.ntiles ? p.ncell : p.ntiles;
  hipLaunchKernelGGL(k_prep, dim3(blocks(n, 256)), dim3(256), 0, c->astream, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  BrickBinArgs b;
  b.N = c->p.n_atoms;
  b.g = atom_geo(c);
  b.nb0 = c->geo.nb[0];
  b.nb1 = c->geo.nb[1];
  b.x0 = (const float*)(c->ws + c->lay.x0);
  b.d = (const float*)(c->ws + c->lay.disp[c->dcur]);
  b.brick_count = (int*)(c->ws + c->lay.brick_count[par]);
  b.brick_list = (int*)(c->ws + c->lay.brick_list[par]);
  b.cell_count = p.cell_count;
  b.cell_rec = (int4*)(c->bin + c->lay.cell_rec);
  b.err = (uint32_t*)(c->ws + c->lay.err);
  hipLaunchKernelGGL(k_brick_bin, dim3(blocks8(b.N, 256)), dim3(256), 0, c->astream, b);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  CompactArgs a;
  a.cell_count = p.cell_count;
  a.ncell = c->geo.ncell;
  a.occ_cells = (int*)(c->bin + c->lay.occ_cells);
  a.tile_flag = (const uint32_t*)b.brick_count;
  a.ntiles = (int)c->geo.nbricks;
  a.occ_tiles = (int*)(c->ws + c->lay.hot_bricks[par]);
  a.occ_count = p.occ_count;
  const long nb = (a.ncell + 255) / 256 + (a.ntiles + 255) / 256;
  hipLaunchKernelGGL(k_compact, dim3((unsigned)nb), dim3(256), 0, c->astream, a);
  return hipGetLastError();
}

hipError_t launch_cell_sort(lb_ctx* c) {
  SortArgs a;
  a.occ_cells = (const int*)(c->bin + c->lay.occ_cells);
  a.occ_count = (const int*)(c->bin + c->lay.occ_count[c->step & 1]);
  a.cell_count = (const int*)(c->bin + c->lay.cell_count);
  a.cell_rec = (int4*)(c->bin + c->lay.cell_rec);
  hipLaunchKernelGGL(k_cell_sort, dim3(persistent_grid(std::min(c->geo.ncell, (long)c->p.n_atoms))),
                     dim3(256), 0, c->astream, a);
  return hipGetLastError();
}

hipError_t launch_bin_mark(lb_ctx* c) {
  BinArgs a;
  a.N = c->p.n_atoms;
  a.g = atom_geo(c);
  a.x0 = (const float*)(c->ws + c->lay.x0);
  a.d = (const float*)(c->ws + c->lay.disp[c->dcur]);
  const int par = (int)(c->step & 1);
  a.tile_flag = (uint32_t*)(c->bin + c->lay.tile_flag[par]);
  a.node_flag = (uint8_t*)(c->ws + c->lay.node_flag);
  a.base_count = (int*)(c->bin + c->lay.base_count[par]);
  a.base_list = (int*)(c->bin + c->lay.base_list[par]);
  a.atom_frac = (float4*)(c->bin + c->lay.atom_frac);
  a.cell_count = (int*)(c->bin + c->lay.cell_count);
  a.cell_rec = (int4*)(c->bin + c->lay.cell_rec);
  a.err = (uint32_t*)(c->ws + c->lay.err);
  hipLaunchKernelGGL(k_bin_mark, dim3(blocks8(a.N, 256)), dim3(256), 0, c->astream, a);
  return hipGetLastError();
}

hipError_t launch_node_u(lb_ctx* c) {
  const Geometry& g = c->geo;
  NodeArgs a;
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
  a.node_list = (const int*)(c->bin + c->lay.node_list[c->step & 1]);
  a.node_count = (const int*)(c->bin + c->lay.occ_count[c->step & 1]) + 2;
  a.uc = (float*)(c->bin + c->lay.uc);
  a.dnx = g.div_nx;
  a.dny = g.div_ny;
  a.narrow = g.narrow ? 1 : 0;
  const dim3 grid(node_grid(c)), block(256);
  const bool q27 = c->geo.q == 27;
  switch (c->p.storage) {
    case LB_STORE_F32:
      if (q27) hipLaunchKernelGGL((k_node_u<LB_STORE_F32, 27>), grid, block, 0, c->stream, a);
      else hipLaunchKernelGGL((k_node_u<LB_STORE_F32, 19>), grid, block, 0, c->stream, a);
      break;
    case LB_STORE_F16:
      if (q27) hipLaunchKernelGGL((k_node_u<LB_STORE_F16, 27>), grid, block, 0, c->stream, a);
      else hipLaunchKernelGGL((k_node_u<LB_STORE_F16, 19>), grid, block, 0, c->stream, a);
      break;
    default:
      if (q27) hipLaunchKernelGGL((k_node_u<LB_STORE_BF16, 27>), grid, block, 0, c->stream, a);
      else hipLaunchKernelGGL((k_node_u<LB_STORE_BF16, 19>), grid, block, 0, c->stream, a);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_couple(lb_ctx* c) {
  CoupleArgs a;
  a.N = c->p.n_atoms;
  a.n[0] = c->geo.nx;
  a.n[1] = c->geo.ny;
  a.n[2] = c->geo.nz;
  a.plane = c->geo.plane;
  a.gamma = c->p.gamma;
  a.x0 = (const float*)(c->ws + c->lay.x0);
  a.d = (const float*)(c->ws + c->lay.disp[c->dcur]);
  a.v = (const float*)(c->ws + c->lay.vel);
  a.uc = (const float*)(c->bin + c->lay.uc);
  a.fc = (float*)(c->bin + c->lay.fc);
  a.U = c->couple_u;
  hipLaunchKernelGGL(k_couple, dim3(blocks8(8L * a.N, 256)), dim3(256), 0, c->stream, a);
  return hipGetLastError();
}

hipError_t launch_spread(lb_ctx* c) {
  SpreadArgs a;
  a.S = (int)c->geo.S;
  a.n[0] = c->geo.nx;
  a.n[1] = c->geo.ny;
  a.n[2] = c->geo.nz;
  a.plane = c->geo.plane;
  const int par = (int)(c->step & 1);
  a.node_list = (const int*)(c->bin + c->lay.node_list[par]);
  a.node_count = (const int*)(c->bin + c->lay.occ_count[par]) + 2;
  a.node_flag = (uint8_t*)(c->ws + c->lay.node_flag);
  a.base_count = (const int*)(c->bin + c->lay.base_count[par]);
  a.base_list = (const int*)(c->bin + c->lay.base_list[par]);
  a.atom_frac = (const float4*)(c->bin + c->lay.atom_frac);
  a.fc = (const float*)(c->bin + c->lay.fc);
  a.fcoup = (float*)(c->bin + c->lay.fcoup[par]);
  hipLaunchKernelGGL(k_spread, dim3(node_grid(c)), dim3(256), 0, c->stream, a);
  return hipGetLastError();
}

static ForceArgs force_args(lb_ctx* c) {
  ForceArgs a;
  a.N = c->p.n_atoms;
  a.g = atom_geo(c);
  a.ncell = c->geo.ncell;
  for (int k = 0; k < 3; ++k) {
    a.L[k] = (float)a.g.n[k];
    a.invL[k] = 1.0f / (float)a.g.n[k];
  }
  a.x0 = (const float*)(c->ws + c->lay.x0);
  a.d = (const float*)(c->ws + c->lay.disp[c->dcur]);
  a.ff = (float*)(c->ws + c->lay.ff);
  a.k_tether = c->p.k_tether;
  a.bond_off = (const int*)(c->ws + c->lay.bond_off);
  a.bond_nbr = (const int*)(c->ws + c->lay.bond_nbr);
  a.k_bond = c->p.k_bond;
  a.r0_bond = c->p.r0_bond;
  a.lj_eps24 = 24.0f * c->p.lj_eps;
  a.lj_sigma2 = c->p.lj_eps != 0.0f ? c->p.lj_sigma * c->p.lj_sigma : 0.0f;
  a.coul2 = 2.0f * c->p.coul_k;
  a.charge = (const float*)(c->ws + c->lay.charge);
  a.lj_rc2 = c->p.lj_rc * c->p.lj_rc;
  a.lj_exclude_bonded = c->p.lj_exclude_bonded;
  a.cell_count = (const int*)(c->bin + c->lay.cell_count);
  a.cell_rec = (const int4*)(c->bin + c->lay.cell_rec);
  a.occ_cells = (const int*)(c->bin + c->lay.occ_cells);
  a.occ_count = (const int*)(c->bin + c->lay.occ_count[c->step & 1]);
  a.err = (uint32_t*)(c->ws + c->lay.err);
  a.lf = nullptr;
  a.lx_in = nullptr;
  a.lx_out = nullptr;
  return a;
}

// Workgroups of the force field.  Started after the coupling kernels, it runs beside the spread
// and the sweep, and 512 (2 wavefronts per SIMD) leave the sweep room: per step at 256^3 with
// 200k atoms 0.557 ms against 0.566 (768), 0.599 (1024) and 0.635 (256); at 384^3 with 1M atoms
// 2.085 ms against 2.125, 2.259 and 2.492.  Started right after the cell sort beside a short
// 16-bit sweep, it is on the longer cycle, and 768 gain about 1% (FP16 at 256^3: 0.361 against
// 0.365 ms; at 384^3: 1.428 against 1.447).  Alone on one stream it takes the whole persistent
// grid (2048 at most).
static unsigned force_grid_cap(const lb_ctx* c) {
  if (c->astream == c->stream) return 2048u;
  return c->geo.late_forces ? 512u : 768u;
}

hipError_t launch_forces(lb_ctx* c) {
  const ForceArgs a = force_args(c);
  const dim3 grid(std::min(persistent_grid(std::min(a.ncell, (long)a.N)), force_grid_cap(c)));
  if (a.ncell > 0 && a.coul2 != 0.f)
    hipLaunchKernelGGL((k_forces_cells<false, true>), grid, dim3(256), 0, c->astream, a);
  else if (a.ncell > 0)
    hipLaunchKernelGGL((k_forces_cells<false, false>), grid, dim3(256), 0, c->astream, a);
  else
    hipLaunchKernelGGL(k_bonded_forces<false>, dim3(blocks(a.N, 256)), dim3(256), 0, c->astream, a);
  return hipGetLastError();
}

hipError_t launch_force_hvp(lb_ctx* c, const float4* lf, const float* lx_in, float* lx_out, hipStream_t st) {
  ForceArgs a = force_args(c);
  a.lf = lf;
  a.lx_in = lx_in;
  a.lx_out = lx_out;
  const dim3 grid(persistent_grid(std::min(a.ncell, (long)a.N)));
  if (a.ncell > 0 && a.coul2 != 0.f)
    hipLaunchKernelGGL((k_forces_cells<true, true>), grid, dim3(256), 0, st, a);
  else if (a.ncell > 0)
    hipLaunchKernelGGL((k_forces_cells<true, false>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL(k_bonded_forces<true>, dim3(blocks(a.N, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_integrate(lb_ctx* c) {
  IntegrateArgs a;
  a.N = c->p.n_atoms;
  a.inv_mass = 1.0f / c->p.mass;
  a.ff = (const float*)(c->ws + c->lay.ff);
  a.fc = (const float*)(c->bin + c->lay.fc);
  a.d = (const float*)(c->ws + c->lay.disp[c->dcur]);
  a.d_next = (float*)(c->ws + c->lay.disp[c->dcur ^ 1]);
  a.v = (float*)(c->ws + c->lay.vel);
  a.err = (uint32_t*)(c->ws + c->lay.err);
  hipLaunchKernelGGL(k_integrate, dim3(blocks(a.N, 256)), dim3(256), 0, c->astream, a);
  return hipGetLastError();
}

hipError_t launch_read_atoms(lb_ctx* c, float* x, float* v) {
  const int N = c->p.n_atoms;
  hipLaunchKernelGGL(k_read_atoms, dim3(blocks(3L * N, 256)), dim3(256), 0, c->stream, N,
                     (const float*)(c->ws + c->lay.x0), (const float*)(c->ws + c->lay.disp[c->dcur]),
                     (const float*)(c->ws + c->lay.vel), x, v);
  return hipGetLastError();
}

}  // namespace lbmd
