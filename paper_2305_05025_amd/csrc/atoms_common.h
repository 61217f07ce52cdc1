// Device and launch helpers shared by the atom-side kernels of the forward step and of its
// adjoint: positions as anchor + displacement, stencil and neighbour-list cell geometry,
// fixed-point conversions, XCD-aware workgroup numbering and grid sizes.
#pragma once

#include "lattice_common.h"

namespace lbmd {

__device__ __forceinline__ int wrapi(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// The atoms' displacement d = X - x0 and velocity v are float-float pairs, hi + lo: hi is the
// value rounded to FP32 and lo the remainder, so the integrator accumulates them exactly and
// every use rounds once from the exact sum instead of carrying the rounding of every earlier
// step.  The arrays hold all hi parts [N][3], then all lo parts [N][3].
//
// s + e = a + b exactly (Knuth's two-sum; needs round-to-nearest and no reassociation)
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// (hi, lo) + (b_hi, b_lo) renormalised so that hi is the sum rounded to FP32
__device__ __forceinline__ void ff_add(float& hi, float& lo, float b_hi, float b_lo) {
  float s, e;
  two_sum(hi, b_hi, s, e);
  const float t = (lo + b_lo) + e;
  hi = s + t;
  lo = t - (hi - s);
}

// Integer node and fraction of X = x0 + (d_hi + d_lo) along one axis, the node wrapped into
// [0, n).  The fraction is formed from the exact sum of the anchor's fraction and d_hi plus
// d_lo, so it keeps FP32 resolution however far the atom has moved.  The clamp keeps a
// diverging displacement (reported by the velocity check) from producing out-of-range integer
// conversions.
__device__ __forceinline__ void split(float x0, float d_hi, float d_lo, int n, int& i0,
                                      float& frac) {
  const float ia = floorf(x0);
  float s, e;
  two_sum(x0 - ia, fminf(fmaxf(d_hi, -1.0e6f), 1.0e6f), s, e);
  float fl = floorf(s);
  float r = (s - fl) + (e + d_lo);   // s - fl is exact
  if (r < 0.0f) {
    r += 1.0f;
    fl -= 1.0f;
  }
  if (r >= 1.0f) {   // also a negative r whose sum with 1 rounded up to 1
    r -= 1.0f;
    fl += 1.0f;
  }
  frac = r;
  i0 = wrapi((int)ia + (int)fl, n);
}

// Neighbour-list cell of a wrapped position, and the integer origin of that cell.
__device__ __forceinline__ int cell_of(int i0, float frac, float inv_cw, int nc) {
  const int q = (int)(((float)i0 + frac) * inv_cw);
  return q >= nc ? nc - 1 : q;
}
__device__ __forceinline__ int cell_origin(int q, int n, int nc) { return (q * n) / nc; }

// Position of an atom inside its neighbour-list cell in 8.24 fixed point: (node offset from
// the cell's integer origin, biased by 1) + fraction.  Differences of these integers are
// exact, and one conversion turns a pair difference into a float.
constexpr float kCellFix = 16777216.0f;      // 2^24
constexpr float kCellFixInv = 1.0f / 16777216.0f;
__device__ __forceinline__ int cell_fixed(int node_offset, float frac) {
  return ((node_offset + 1) << 24) + (int)rintf(frac * kCellFix);
}

// value * scale rounded to an integer, clamped so a diverging state (which the velocity
// check reports) cannot overflow the conversion
__device__ __forceinline__ long long to_fixed(float v, float scale) {
  float q = rintf(v * scale);
  q = fminf(fmaxf(q, -4.0e18f), 4.0e18f);
  return (long long)q;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.  Kernels whose
// neighbouring work items share data (atoms of one globule, nodes of one region) renumber
// their workgroups so that each XCD gets one contiguous eighth of the grid.  The grid must be
// a multiple of 8 workgroups.
__device__ __forceinline__ int xcd_block() {
  const int per = (int)(gridDim.x >> 3);
  return (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
}


struct AtomGeo {
  int n[3];          // lattice extents
  int nc[3];         // neighbour-list cells per axis (nc[0] == 0: no Lennard-Jones)
  float inv_cw[3];
};

__device__ __forceinline__ float min_image(float r, float L, float invL) {
  return r - L * rintf(r * invL);
}

// per-axis neighbour-cell index after periodic wrap, and the integer shift (own cell origin
// minus neighbour cell origin, across the periodic seam if it wrapped) that expresses the
// neighbour's cell-relative positions in the own cell's frame
__device__ __forceinline__ void nbr_cell(int q, int o, int n, int nc, int& cq, int& shift) {
  int c = q + o, s = 0;
  if (c < 0) {
    c += nc;
    s = n;
  }
  if (c >= nc) {
    c -= nc;
    s = -n;
  }
  cq = c;
  shift = cell_origin(q, n, nc) - cell_origin(c, n, nc) + s;
}

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

inline AtomGeo atom_geo(const lb_ctx* c) {
  AtomGeo g;
  const int n3[3] = {c->geo.nx, c->geo.ny, c->geo.nz};
  for (int k = 0; k < 3; ++k) {
    g.n[k] = n3[k];
    g.nc[k] = c->geo.nc[k];
    g.inv_cw[k] = c->geo.inv_cw[k];
  }
  return g;
}

inline unsigned blocks(long n, int per) { return (unsigned)((n + per - 1) / per); }

// grids of the XCD-mapped kernels are a multiple of 8 workgroups
inline unsigned blocks8(long n, int per) { return (blocks(n, per) + 7u) & ~7u; }

// persistent kernels: enough 4-wavefront workgroups for the items (one per wavefront), at
// most 8 per CU
// one thread per flagged node: enough workgroups for the most nodes there can be (8 per atom,
// at most one per site), at most 2048
inline unsigned node_grid(const lb_ctx* c) {
  const long n = std::min(8L * c->p.n_atoms, (long)c->geo.S);
  const long b = (n + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

inline unsigned persistent_grid(long nitems) {
  long b = (nitems + 3) / 4;
  if (b > 2048) b = 2048;
  if (b < 8) b = 8;
  return (unsigned)((b + 7) & ~7L);
}

}  // namespace lbmd
