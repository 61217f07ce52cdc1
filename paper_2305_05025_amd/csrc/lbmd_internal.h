// Internal declarations of the gfx950 coupled lattice-Boltzmann / atom library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "lbmd.h"

namespace lbmd {

// Lattice velocities in the ordering published by lb_velocity_set_q(): the first 19 are the
// D3Q19 set named after Eq. 1 of the paper, the last 8 the corners that complete D3Q27 (the
// higher-order set of the paper's outlook, Section 4).  opposite(i) = i + 1 for odd i.
constexpr int CX[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                        1, -1, 1, -1, 1, -1, -1, 1};
constexpr int CY[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                        1, -1, 1, -1, -1, 1, 1, -1};
constexpr int CZ[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                        1, -1, -1, 1, 1, -1, 1, -1};
// D3Q19 weights (also those of the thermal-noise moment basis and of the adjoint)
constexpr float WQ[19] = {
    1.f / 3.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f, 1.f / 18.f,
    1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f,
    1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
// D3Q27 weights: 8/27 rest, 2/27 faces, 1/54 edges, 1/216 corners
constexpr float WQ27[27] = {
    8.f / 27.f, 2.f / 27.f, 2.f / 27.f, 2.f / 27.f, 2.f / 27.f, 2.f / 27.f, 2.f / 27.f,
    1.f / 54.f, 1.f / 54.f, 1.f / 54.f, 1.f / 54.f, 1.f / 54.f, 1.f / 54.f,
    1.f / 54.f, 1.f / 54.f, 1.f / 54.f, 1.f / 54.f, 1.f / 54.f, 1.f / 54.f,
    1.f / 216.f, 1.f / 216.f, 1.f / 216.f, 1.f / 216.f,
    1.f / 216.f, 1.f / 216.f, 1.f / 216.f, 1.f / 216.f};
// weight of velocity i in the Q-velocity set (Q = 19 or 27)
template <int Q>
constexpr float wq(int i) { return Q == 27 ? WQ27[i] : WQ[i]; }

constexpr int kSweepBlock = 256;        // sites per sweep workgroup
constexpr int kTileShift = 6;           // force tile = 64 sites (one wavefront of the sweep)
// Per-site planes (populations, forces, flags) start kPlanePad elements apart beyond the
// site count rounded to 64: with a power-of-two lattice the 19 population planes would
// otherwise share every low address bit, and the sweep's 38 streams measured about 1% slower.
constexpr long kPlanePad = 256;
// Bricks of 16 x 4 x 4 sites (one sweep workgroup each): the unit of the coupled part of the
// sweep.  A brick that some atom's 2 x 2 x 2 stencil touches is "hot": one workgroup computes
// the coupling velocity on the brick and a one-node halo, the friction of the atoms listed
// there and their spread force, and updates the brick's sites; the other sites are swept
// plainly.
constexpr int kBrickX = 16, kBrickY = 4, kBrickZ = 4;
constexpr int kBrickShiftX = 4, kBrickShiftY = 2, kBrickShiftZ = 2;
constexpr int kHaloX = kBrickX + 2, kHaloY = kBrickY + 2, kHaloZ = kBrickZ + 2;
constexpr int kHaloNodes = kHaloX * kHaloY * kHaloZ;   // 648
// atoms listed per brick: those whose stencil base lies in the 17 x 5 x 5 nodes around it
// (at most 425 for atoms at least one lattice spacing apart along some axis); more latches
// LB_EOVERFLOW
constexpr int kBrickCap = 640;
constexpr int kCellCap = 48;            // atoms per neighbour-list cell
constexpr int kBaseCap = 8;             // atoms whose stencil base is one node
constexpr float kFixScale = 1099511627776.0f;      // 2^40: fixed-point scale of spread forces
constexpr float kFixInv = 1.0f / 1099511627776.0f;

// latched device-side conditions (bits of err[0])
constexpr uint32_t kErrOverflow = 1u;
constexpr uint32_t kErrNonFinite = 2u;

// Byte offsets of every buffer.  The buffers a step's binning and coupling produce (from
// fcoup to cell_rec, and U) are offsets into the binning region at lb_ctx::bin, normally the
// part of the workspace at bin_base; the adjoint gives each step of a segment a region of its
// own, so that its backward step reuses the binning of its recomputed forward step.  All
// others are offsets into the workspace.
struct Layout {
  size_t pop[2];       // population buffers A / B, q planes of `plane` elements
  size_t bin_base;     // the binning region inside the workspace, and its size
  size_t bin_bytes;
  // [step parity]: a step's sweep still reads these while the next step bins its atoms
  size_t fcoup[2];     // float [3][plane]: spread coupling force at marked nodes
  size_t tile_flag[2]; // uint32 per 64-site force tile
  size_t base_count[2];// int32 [plane]: atoms whose stencil base (lower corner) is this node
  size_t base_list[2]; // int32 [plane][kBaseCap]
  size_t node_flag;    // uint8 [plane]: atom stencil nodes of this step
  size_t uc;           // float [3][plane]: coupling velocity at marked nodes
  size_t atom_frac;    // float4 [N]: stencil fractions of each atom
  size_t occ_cells;    // int32 [min(ncell, N)]: neighbour-list cells holding atoms this step
  size_t occ_tiles[2]; // int32 [ntiles]: flagged force tiles, by step parity
  size_t node_list[2]; // int32 [min(8 N, S)]: flagged nodes (atom stencil nodes), by step parity
  size_t occ_count[2]; // int32 [4] by step parity: lengths of the cell, tile (or hot-brick)
                       // and node lists
  size_t brick_count[2]; // int32 [nbricks] by step parity: atoms listed per brick
  size_t brick_list[2];  // int32 [nbricks][kBrickCap]
  size_t hot_bricks[2];  // int32 [nbricks]: the hot bricks, compacted
  size_t fext_tab;     // float [ny]   (Kolmogorov / sign-shear profile)
  size_t fext_field;   // float [3][plane] (caller field)
  size_t x0;           // float [N][3] anchors
  size_t disp[2];      // float [2][N][3] displacement X - x0 (hi, lo), double-buffered
  size_t vel;          // float [2][N][3] velocity (hi, lo)
  size_t fc;           // float [N][3] friction force of the current step
  size_t ff;           // float [N][3] stand-in force field at X^n
  size_t charge;       // float [N] atom charges (Coulomb term)
  size_t bond_off;     // int32 [N+1]
  size_t bond_nbr;     // int32 [2 n_bonds]
  size_t cell_count;   // int32 [ncell]
  size_t cell_rec;     // int4 [ncell][kCellCap]: fixed-point position in the cell, atom index
  size_t U;            // float [N][3]: fluid velocity interpolated at each atom (adjoint only)
  size_t red_partial;  // double [kRedBlocks][4]
  size_t red_out;      // double [8]
  size_t err;          // uint32 [4]
  size_t total;
};

// Division by a run-time invariant divisor d >= 1 with a multiply-high, an add and a shift
// (Granlund and Montgomery, "Division by invariant integers using multiplication", PLDI 1994,
// Section 4): with l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
// floor(n / d) = (mulhi(n, m) + n) >> l for every 0 <= n < 2^32 whose sum does not overflow,
// so for all n < 2^31 (site indices).
struct FastDiv {
  uint32_t m;
  uint32_t l;
};
inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  return {(uint32_t)m, l};
}

constexpr int kRedBlocks = 1024;
// the fixed scratch of lb_invariants_noalloc: kRedBlocks partial sums of 4 doubles (32 KiB)
constexpr int kNoallocScratchDoubles = kRedBlocks * 4;
constexpr int kTimedEvents = 8;

struct Geometry {
  int q;             // lattice velocities: 19 or 27
  int nx, ny, nz;
  long S;            // sites
  long plane;        // population plane stride (elements), S rounded up to 64 plus kPlanePad
  int nblocks;       // ceil(S / kSweepBlock)
  int ntiles;        // ceil(S / 64): force tiles
  int nb[3];         // bricks per axis
  long nbricks;
  int nc[3];         // neighbour-list cells per axis (0 when LJ is off)
  long ncell;
  float inv_cw[3];   // 1 / cell width
  size_t elem;       // bytes per stored population value
  FastDiv div_nx, div_ny;  // site index -> (x, y, z)
  // Every population plane's sites fit in 4 GiB (S * elem <= 2^32): the lattice kernels then
  // address a plane by a scalar base and a 32-bit lane byte offset.  Setting the environment
  // variable LBMD_WIDE_OFFSETS (any value) at context creation keeps the 64-bit addressing
  // that larger lattices take, so both forms can be compared on small ones.
  bool narrow;
  // In the two-stream step, the force field waits for the coupling kernels when the sweep is
  // long: at least 2^23 sites, and at least 7 KiB of population traffic per step and atom
  // (FP32 D3Q19 at 256^3 with 200k atoms moves 12.5 KiB, at 384^3 with 1M atoms 8.4 KiB; FP16
  // at 256^3 with 200k atoms 6.2 KiB).  Otherwise it starts right after the cell sort.  The
  // environment variable LBMD_LATE_FORCES (any value) at context creation takes the late start
  // on any lattice, so both orders can be compared on small ones.
  bool late_forces;
  // LB_FLAG_FUSED_COUPLING with atoms: the coupled step runs as the hot-brick sweep beside the
  // cold sweep; otherwise the coupling velocity, friction and spread run as separate kernels
  // before one sweep over every site.  Both give the same bits.
  bool fused;
  // The atom work runs on a stream of its own beside the lattice stream: atoms present, no
  // LB_FLAG_SINGLE_STREAM, and more than LB_ONE_STREAM_MAX_SITES sites.  The environment
  // variable LBMD_OVERLAP_SMALL (any value) at context creation lifts the size limit, so the
  // two schedules can be compared on small lattices.
  bool overlap;
};

bool geometry(const lb_params* p, Geometry* g);
Layout plan(const lb_params* p, const Geometry& g);
// Offsets of the binning region's buffers (relative to its start) into *l; returns its size.
// one_parity: a region used by one step only, whose [2] buffers share one allocation.
size_t plan_bin(const lb_params* p, const Geometry& g, bool one_parity, Layout* l);

}  // namespace lbmd

struct lb_ctx {
  lb_params p;
  lbmd::Geometry geo;
  lbmd::Layout lay;
  hipStream_t stream;
  int device;       // the HIP device current at lb_init
  char* ws;
  char* bin;        // the binning region (inside ws; the adjoint points it at a step's own)
  char* popbuf[2];  // population buffers A / B (inside ws; the adjoint points them at its slots)
  float* couple_u = nullptr;  // when set, k_couple also stores U (the adjoint needs it)
  // the sweep leaves the spread force and the base-node counts in place (the adjoint's
  // recomputed steps, whose backward steps read them)
  bool keep_coupling = false;
  int cur;        // which population buffer holds the current state
  int dcur;       // which displacement buffer holds X^n - x0
  int64_t step;
  float omega;    // 1 / tau
  float omega_m;  // rate of the odd part under the two-relaxation-time collision (= omega for BGK)
  std::string err;
  // second stream for the atom work that overlaps the sweep, and its fork/join events
  hipStream_t astream = nullptr;  // atom stream (the caller's stream when single-stream)
  hipEvent_t ev_fork = nullptr, ev_bin = nullptr, ev_couple = nullptr, ev_spread = nullptr, ev_join = nullptr;
  // fused step: the hot-brick sweep runs on a stream of its own beside the cold sweep; events
  // by step parity (a wait refers to the previous step's record while this step's is queued)
  hipStream_t hstream = nullptr;
  hipEvent_t ev_hot[2] = {nullptr, nullptr}, ev_cold[2] = {nullptr, nullptr};
  // LB_FLAG_STEP_GRAPHS: the two-step graph of each starting parity (built on first use) and
  // the stream it is captured on
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipStream_t gstream = nullptr;
  // optional per-phase event timing (lb_timing_begin / lb_timing_end)
  std::vector<hipEvent_t> ev;  // kTimedEvents per timed step
  int timed_cap = 0;
  int timed = 0;
};

namespace lbmd {

// ---- kernel launchers (lb_sweep.hip) ----
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_copy_pair(void* d0, const void* s0, void* d1, const void* s1, size_t bytes,
                            hipStream_t s);
hipError_t launch_sweep(lb_ctx* c, const void* fin, void* fout, hipStream_t st);
// the two parts of the coupled sweep: the hot bricks (coupling + update of their sites), then
// every other site
hipError_t launch_hot_sweep(lb_ctx* c, const void* fin, void* fout, hipStream_t st);
hipError_t launch_cold_sweep(lb_ctx* c, const void* fin, void* fout, hipStream_t st);
hipError_t launch_read_fields(lb_ctx* c, float* rho, float* u);
hipError_t launch_read_populations(lb_ctx* c, float* g);
hipError_t launch_write_populations(lb_ctx* c, const float* g);
// the FP64 sums of the current state: per-workgroup partials (invariants_blocks(c) x 4
// doubles) into `partial`, the 7 results into `out` (device pointers)
int invariants_blocks(const lb_ctx* c);
hipError_t launch_invariants(lb_ctx* c, double* partial, double* out);
// lb_invariants_noalloc's scratch: looked up once per device (with that device current),
// then its device address on `device` (NULL before set-up)
hipError_t setup_invariants_scratch(int device);
double* invariants_scratch(int device);
hipError_t launch_store_i64(void* dst, int64_t v, hipStream_t s);

// ---- kernel launchers (atoms.hip) ----
hipError_t launch_prep(lb_ctx* c);
hipError_t launch_bin_mark(lb_ctx* c);
hipError_t launch_compact(lb_ctx* c);   // occupied cells, flagged tiles, then flagged nodes
hipError_t launch_cell_sort(lb_ctx* c);
// binning of the fused path: atoms to the bricks their stencils touch and to the neighbour-list
// cells; lists of the hot bricks and of the occupied cells
hipError_t launch_brick_binning(lb_ctx* c);
hipError_t launch_node_u(lb_ctx* c);
hipError_t launch_couple(lb_ctx* c);
hipError_t launch_spread(lb_ctx* c);
hipError_t launch_forces(lb_ctx* c);
// adjoint: lx_out = lx_in + (d F_ff / d X)^T lf at the context's current positions
hipError_t launch_force_hvp(lb_ctx* c, const float4* lf, const float* lx_in, float* lx_out, hipStream_t st);
hipError_t launch_integrate(lb_ctx* c);
hipError_t launch_read_atoms(lb_ctx* c, float* x, float* v);

// ---- adjoint (adjoint.hip) ----
// Buffers of one adjoint step: "in" holds the adjoints at step n + 1, "out" receives them at
// step n.  U is the interpolated fluid velocity that k_couple stored for this step.
struct AdjointBuffers {
  const float* lam_in;   // dL/dP^{n+1}, FP32 [19][plane]
  float* lam_out;        // dL/dP^n
  float* phi;            // [3][plane] dL/dF on flagged tiles
  float* luc;            // [3][plane] dL/du_c on flagged tiles
  float* db;             // [3][S] dL/dF_ext accumulated, or NULL
  double* dom_part;      // [2][nblocks]: dL/domega+, dL/domega- per workgroup
  double* dg_part;       // [adjoint_atom_blocks]
  double* acc;           // [3]: dL/dgamma, dL/domega+, dL/domega-
  const float* U;        // [N][3]
  float* lU;             // [N][3]
  float4* lf;            // [N]
  const float* lx_in;    // [N][3] dL/dX^{n+1}
  const float* lv_in;    // [N][3] dL/dv^{n+1}
  float* lx_out;
  float* lv_out;
  float* lxa;            // [N][3] the coupling's part of dL/dX^n (scratch of the step)
  // the force field's Hessian-vector product runs on `side` beside the lattice part when it
  // is set and differs from the context's stream, forked and joined with the two events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};
unsigned adjoint_atom_blocks(const lb_ctx* c);
// the adjoint of step c->step, with the context's forward buffers holding that step's
// binning, coupling velocity, friction and spread force
hipError_t launch_adjoint_step(lb_ctx* c, const AdjointBuffers& b);

}  // namespace lbmd
