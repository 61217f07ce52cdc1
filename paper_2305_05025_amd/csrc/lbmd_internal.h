// Internal declarations of the gfx950 coupled lattice-Boltzmann / atom library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lbmd.h"

namespace lbmd {

// D3Q19 lattice (the 19-speed set named after Eq. 1 of the paper): velocities and weights,
// in the ordering published by lb_velocity_set().
constexpr int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr float WQ[19] = {
    1.f / 3.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f,
    1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
    1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};

constexpr int kSweepBlock = 256;        // sites per sweep workgroup = sites per force tile
constexpr int kTileShift = 8;           // log2(kSweepBlock)
constexpr int kCellCap = 48;            // atoms per neighbour-list cell
constexpr float kFixScale = 1099511627776.0f;      // 2^40: fixed-point scale of spread forces
constexpr float kFixInv = 1.0f / 1099511627776.0f;

// latched device-side conditions (bits of err[0])
constexpr uint32_t kErrOverflow = 1u;
constexpr uint32_t kErrNonFinite = 2u;

// Byte offsets of every buffer inside the caller's workspace.
struct Layout {
  size_t pop[2];       // population buffers A / B, 19 planes of `plane` elements
  size_t fcoup;        // spread coupling force, fixed point int64 [3][plane]
  size_t tile_flag;    // uint32 per force tile
  size_t fext_tab;     // float [ny]   (Kolmogorov / sign-shear profile)
  size_t fext_field;   // float [3][plane] (caller field)
  size_t x0;           // float [N][3] anchors
  size_t disp[2];      // float [N][3] displacement X - x0, double-buffered
  size_t vel;          // float [N][3]
  size_t fc;           // float [N][3] friction force of the current step
  size_t bond_off;     // int32 [N+1]
  size_t bond_nbr;     // int32 [2 n_bonds]
  size_t cell_count;   // int32 [ncell]
  size_t cell_atoms;   // int32 [ncell][kCellCap]
  size_t red_partial;  // double [kRedBlocks][4]
  size_t red_out;      // double [8]
  size_t err;          // uint32 [4]
  size_t total;
};

constexpr int kRedBlocks = 1024;

struct Geometry {
  int nx, ny, nz;
  long S;            // sites
  long plane;        // population plane stride (elements), S rounded up to 64
  int ntiles;        // ceil(S / kSweepBlock)
  int nc[3];         // neighbour-list cells per axis (0 when LJ is off)
  long ncell;
  float inv_cw[3];   // 1 / cell width
  size_t elem;       // bytes per stored population value
};

bool geometry(const lb_params* p, Geometry* g);
Layout plan(const lb_params* p, const Geometry& g);

}  // namespace lbmd

struct lb_ctx {
  lb_params p;
  lbmd::Geometry geo;
  lbmd::Layout lay;
  hipStream_t stream;
  char* ws;
  int cur;        // which population buffer holds the current state
  int dcur;       // which displacement buffer holds X^n - x0
  int64_t step;
  float omega;    // 1 / tau
  std::string err;
  // optional per-phase event timing (lb_timing_begin / lb_timing_end)
  std::vector<hipEvent_t> ev;  // 4 per timed step: atoms begin/end, sweep begin/end
  int timed_cap = 0;
  int timed = 0;
};

namespace lbmd {

// ---- kernel launchers (lb_sweep.hip) ----
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_sweep(lb_ctx* c, const void* fin, void* fout);
hipError_t launch_read_fields(lb_ctx* c, float* rho, float* u);
hipError_t launch_read_populations(lb_ctx* c, float* g);
hipError_t launch_write_populations(lb_ctx* c, const float* g);
hipError_t launch_invariants(lb_ctx* c);
hipError_t launch_store_i64(void* dst, int64_t v, hipStream_t s);

// ---- kernel launchers (atoms.hip) ----
hipError_t launch_prep(lb_ctx* c);
hipError_t launch_couple(lb_ctx* c);
hipError_t launch_cell_sort(lb_ctx* c);
hipError_t launch_forces_integrate(lb_ctx* c);
hipError_t launch_read_atoms(lb_ctx* c, float* x, float* v);

}  // namespace lbmd
