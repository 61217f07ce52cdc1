/*
 * lbmd.h -- C interface of the MI355X (gfx950) coupled lattice-Boltzmann / atom library.
 *
 * The operation (Lauricella et al., arXiv 2305.05025, Section 2.2):
 *   a periodic D3Q19 lattice (optionally D3Q27, the higher-order velocity set proposed in
 *   Section 4) evolved by the single-relaxation-time (BGK) lattice Boltzmann
 *   equation, Eq. (1), with relaxation time tau = 1/omega = 3 nu + 1/2, the second-order
 *   equilibrium and the moments of Eqs. (2)-(3); atoms coupled to it by a friction force
 *   gamma (u - v), u interpolated linearly over the eight nearest nodes, the opposite force
 *   returned to the lattice through the forcing term S_i of Eq. (1) (Guo scheme) with the
 *   same weights; lattice and atoms advanced in lock-step, one step each.
 *   The atoms' own force field is a stand-in: harmonic tethers to the initial positions,
 *   harmonic bonds, and Lennard-Jones cut off at r_c with minimum image, shifted so that its
 *   force falls continuously to zero at r_c: with the plain term F_i = g0(r^2) r, the force is
 *   (g0(r^2) - g0(r_c^2)) r below r_c and zero beyond (the paper's runs give a cut-off distance
 *   only).
 *
 * Units are lattice units: dx = dt = 1, rest density rho0.  Nodes sit at integer
 * coordinates; positions are continuous.
 *
 * Layouts (all arrays C-contiguous):
 *   site index s = x + nx * (y + ny * z), x fastest; S = nx * ny * nz
 *   scalar field [S], vector field [3][S] (component-major), atom arrays [N][3] float32.
 * Velocity ordering of the Q = 19 (or 27) populations: see lb_velocity_set_q().
 *
 * Ownership: the library never allocates device memory.  The caller provides one device
 * workspace of lb_workspace_bytes() bytes (256-byte aligned) that must stay valid until
 * lb_destroy().  All array arguments are device pointers unless stated; inputs are copied
 * at lb_init, outputs are written into caller buffers.
 *
 * Asynchrony: every call enqueues on the HIP stream given at lb_init (NULL = default
 * stream) and returns without waiting, except lb_init (copies the bond list to the host
 * once), lb_invariants and lb_status_check, which synchronise the stream.
 *
 * Errors: every entry point returns an lb_status.  Arguments are validated before any
 * device work is queued; on failure nothing is queued and lb_last_error() describes why.
 * Device-side conditions (a cell of the neighbour list overflowing, non-finite values)
 * are latched in device memory and reported by the next synchronising call.
 *
 * Threading: a context may be used by one host thread at a time.
 */
#ifndef LBMD_H
#define LBMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_ctx lb_ctx;

typedef enum {
  LB_OK = 0,
  LB_EINVAL = 1,      /* invalid argument (nothing was queued) */
  LB_ENOMEM = 2,      /* workspace too small or misaligned */
  LB_EDEVICE = 3,     /* a HIP runtime call failed */
  LB_ESTATE = 4,      /* call not valid in the context's current state */
  LB_ENONFINITE = 5,  /* a NaN/Inf appeared in the populations or atom velocities */
  LB_EOVERFLOW = 6    /* a neighbour-list cell exceeded its capacity (atoms overlap) */
} lb_status;

/* Storage format of the populations.  All three store the deviation g_i = f_i - w_i rho0
 * (the same scheme written about the rest state); the collision is computed in FP32.
 * Narrow formats round to nearest even on every store. */
typedef enum {
  LB_STORE_F32 = 0,
  LB_STORE_F16 = 1,
  LB_STORE_BF16 = 2
} lb_storage;

/* External force density F_ext(x) entering the forcing term S_i of Eq. (1). */
typedef enum {
  LB_BF_NONE = 0,
  LB_BF_KOLMOGOROV = 1,  /* F_x = amp * sin(2 pi y / ny)                        */
  LB_BF_SIGN_SHEAR = 2,  /* F_x = amp * sign(y + 1/2 - ny/2)                    */
  LB_BF_FIELD = 3        /* F = caller field [3][S] (FP32), copied at lb_init    */
} lb_body_force;

/* lb_params.flags */
#define LB_FLAG_CHECK_FINITE 0x1u  /* lb_couple_step also checks for NaN/Inf every step */
#define LB_FLAG_SINGLE_STREAM 0x2u /* queue every kernel on the caller's stream; by default the
                                      library runs the force field, the integration and the
                                      next step's binning on a stream of its own, where
                                      they overlap the lattice sweep.  Both give identical
                                      bits.  Lattices of at most LB_ONE_STREAM_MAX_SITES
                                      sites always run this schedule: their step is bound
                                      by the host's launch and event calls, and it makes
                                      fewer (32^3 with 500 atoms on MI355X: 0.050 ms per
                                      step against 0.055-0.077 for two streams; from about
                                      2^16 sites on, two streams are as fast or faster) */
#define LB_ONE_STREAM_MAX_SITES 32768u
#define LB_FLAG_FUSED_COUPLING 0x4u /* couple in the sweep itself: every 16 x 4 x 4 brick of sites
                                      that an atom stencil touches is updated by one workgroup
                                      that first computes the coupling velocity on the brick and
                                      its halo, the friction of the atoms there and their spread
                                      force (staged in LDS), on a stream of its own beside the
                                      sweep of the other sites.  Same bits as the default, which
                                      runs the coupling as separate kernels before one sweep.  On
                                      MI355X the default is as fast or faster at every size
                                      measured (256^3 with 200,000 atoms: 0.568 against 0.567 ms
                                      in FP32, 0.364 against 0.408 in FP16; 384^3 with 10^6 atoms
                                      2.13 against 2.44; 32^3 with 500 atoms, both on one stream:
                                      0.050 against 0.067-0.073).  Needs lb_workspace_bytes() for
                                      these flags */
#define LB_FLAG_STEP_GRAPHS 0x8u    /* replay the step from a HIP graph: the first call that starts
                                      at an even (odd) step captures the launches and events of
                                      two steps, and every call of two or more steps replays it,
                                      so the host makes one call per two steps instead of about
                                      sixteen per step.  Same bits as the launches it replaces.
                                      Applies to the unfused step without thermal noise (kT = 0),
                                      without LB_FLAG_CHECK_FINITE and outside lb_timing_begin /
                                      lb_timing_end; other calls, a call's odd last step and the
                                      backward pass's steps are launched as usual.  The graphs
                                      hold the context's buffer addresses and are released by
                                      lb_destroy.  Measured on MI355X it is not faster than the
                                      best eager schedule at any size (ms per step, graphs
                                      against eager two-stream: 32^3 with 500 atoms 0.054
                                      against 0.065, and 0.051 eager on one stream, the default
                                      there; 96^3 0.082
                                      against 0.075; 128^3 0.119 against 0.108; 256^3 0.591
                                      against 0.548): small lattices are bound by the dependent kernels'
                                      dispatch latency on the GPU, which a graph keeps, and the
                                      replay overlaps the atom and lattice work less.  It is for
                                      callers that launch the step from graphs of their own */

typedef struct {
  int32_t L[3];              /* nx, ny, nz >= 2; periodic */
  float tau;                 /* BGK relaxation time, > 0.5: nu = (tau - 1/2)/3 */
  float rho0;                /* rest density, > 0 */
  int32_t storage;           /* lb_storage */
  int32_t n_atoms;           /* >= 0 */
  float mass;                /* atom mass, > 0 when n_atoms > 0 */
  float gamma;               /* friction coefficient (force per unit velocity), >= 0 */
  float k_tether;            /* tether spring to the initial positions; 0 = off */
  int32_t n_bonds;           /* >= 0 */
  float k_bond, r0_bond;     /* harmonic bond U = k/2 (r - r0)^2 */
  float lj_eps, lj_sigma;    /* Lennard-Jones; lj_eps = 0 turns it off */
  float lj_rc;               /* cut-off of the pair terms (force-shifted to zero there);
                                box >= 3 rc per axis */
  int32_t lj_exclude_bonded; /* 1: no LJ between bonded pairs */
  int32_t bf_kind;           /* lb_body_force */
  float bf_amp;
  uint32_t flags;            /* LB_FLAG_* */
  float kT;                  /* thermal energy of the fluctuating-LB noise on the non-conserved
                                modes (Section 2.2, the xi_i of Eq. 1's source term); 0 = off */
  uint32_t seed[2];          /* key of the counter-based (Philox4x32-10) noise generator */
  float coul_k;              /* implicit-solvent Coulomb between atoms (Section 2.2: direct sum,
                                permittivity growing with r): U = coul_k q_i q_j / r^2 under the
                                Lennard-Jones cut-off, shift and exclusions; charges from
                                lb_set_charges (zero until set); 0 = off */
  float trt_magic;           /* collision variant: 0 = BGK (Eq. 1); > 0 = two relaxation times,
                                the part of f - f_eq odd under c -> -c relaxing at omega- with
                                (tau - 1/2)(1/omega- - 1/2) = trt_magic (tau sets the viscosity
                                as before; trt_magic = (tau - 1/2)^2 is BGK again) */
  int32_t velocity_set;      /* lattice velocities: 19 (D3Q19, the set of Eq. 1; 0 also means
                                19) or 27 (D3Q27, the higher-order set of the outlook in
                                Section 4: same equilibrium, forcing and collision over its 27
                                velocities; its thermal noise uses the orthogonal basis of
                                products of the one-dimensional polynomials 1, c, 3c^2 - 1) */
} lb_params;

/* The 19 lattice velocities c[i][0..2] and weights w[i] in the library's ordering:
 * i = 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = (1,1,0),(-1,-1,0),(1,-1,0),(-1,1,0),
 * (1,0,1),(-1,0,-1),(1,0,-1),(-1,0,1),(0,1,1),(0,-1,-1),(0,1,-1),(0,-1,1);
 * opposite(i) = i+1 for odd i.  Weights 1/3, 1/18, 1/36 (the D3Q19 set named after Eq. 1).
 * Host pointers; either may be NULL. */
void lb_velocity_set(int8_t c[19][3], double w[19]);

/* Velocities c[q][3] and weights w[q] of the set with q = 19 (as lb_velocity_set) or 27:
 * the D3Q19 rows in the same order, then the corners i = 19..26 = (1,1,1),(-1,-1,-1),
 * (1,1,-1),(-1,-1,1),(1,-1,1),(-1,1,-1),(-1,1,1),(1,-1,-1) (opposite(i) = i+1 for odd i);
 * D3Q27 weights 8/27, 2/27, 1/54, 1/216 by speed class.  Host pointers; either may be
 * NULL.  LB_EINVAL for any other q. */
lb_status lb_velocity_set_q(int32_t q, int8_t* c, double* w);

/* Bytes of device workspace lb_init needs for these parameters (0 if they are invalid). */
size_t lb_workspace_bytes(const lb_params* p);

/* Create a context and set up the initial state on `hip_stream` (a hipStream_t, NULL for
 * the default stream):
 *   populations at rest equilibrium f_i = w_i rho0 (deviation 0);
 *   atom positions x0 [N][3] (unwrapped lattice coordinates; also the tether anchors and
 *   the origin of the displacement the library integrates), velocities v0 [N][3];
 *   bonds [n_bonds][2] int32 atom index pairs (may be NULL when n_bonds = 0; read back to
 *   the host once to build per-atom bond lists);
 *   body_force [3][S] float32 when bf_kind = LB_BF_FIELD, else ignored.
 * Device pointers.  Inputs are copied; the caller may free them after the call returns.
 * On success *out receives the context. */
lb_status lb_init(const lb_params* p, void* workspace, size_t workspace_bytes,
                  const float* x0, const float* v0, const int32_t* bonds,
                  const float* body_force, void* hip_stream, lb_ctx** out);

/* Advance n_steps >= 0 coupled steps (Section 2.2; one lattice step per atom step).
 * Each step, on the state (g^n pre-collision, X^n, v^n):
 *   1. for every atom, u_c = (j + F_ext/2)/rho at its eight nodes (Eqs. 2-3) and
 *      U = trilinear interpolation of u_c at X^n; friction F_c = gamma (U - v^n);
 *   2. -F_c spread back to the same eight nodes with the same weights;
 *   3. BGK collision with Guo forcing under F = F_ext + spread force, then streaming;
 *   4. atom forces at X^n; v^{n+1} = v^n + (F_ff + F_c)/m, X^{n+1} = X^n + v^{n+1}.
 * Asynchronous. */
lb_status lb_couple_step(lb_ctx* c, int32_t n_steps);

/* Observables of the current state (Eqs. 2-3): rho(x) = rho0 + sum_i g_i,
 * u(x) = (j + F_ext/2)/rho (without the atoms' friction forces), the unwrapped atom
 * positions and velocities.  Device pointers [S], [3][S], [N][3], [N][3]; any may be
 * NULL.  Asynchronous. */
lb_status lb_read_fields(lb_ctx* c, float* rho, float* u, float* x_unwrapped, float* v);

/* Atom displacements X - x0 [N][3] (device pointer): the quantity the library integrates,
 * at full FP32 precision (an unwrapped position x0 + d rounded to FP32 loses the low bits
 * of small displacements).  Asynchronous. */
lb_status lb_read_displacement(lb_ctx* c, float* d);

/* Atom charges q [N] (device, FP32) for the Coulomb term, copied into the context
 * (asynchronous on its stream; the caller's buffer may be reused once the stream has passed
 * this call).  Charges start at zero. */
lb_status lb_set_charges(lb_ctx* c, const float* q);

/* Raw populations of the current pre-collision state as float32 deviations g_i
 * [Q][S] (device pointer, Q = velocity_set), in the lb_velocity_set_q ordering.
 * Asynchronous. */
lb_status lb_read_populations(lb_ctx* c, float* g);

/* Replace the current pre-collision state by caller deviations g [Q][S] (float32, device
 * pointer, lb_velocity_set_q ordering), rounded to the storage format.  Atoms are unchanged.
 * Lets a run start from any lattice state (restart from external data, tests).
 * Asynchronous. */
lb_status lb_set_populations(lb_ctx* c, const float* g);

/* Conserved sums accumulated in FP64 on the device, written to host out7:
 * [0] mass sum_x rho, [1..3] fluid momentum sum_x j, [4..6] atom momentum sum_a m v.
 * Synchronises the stream; returns LB_ENONFINITE / LB_EOVERFLOW if latched. */
lb_status lb_invariants(lb_ctx* c, double out7[7]);

/* For callers that cannot allocate device memory or wait on the stream (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sums of lb_invariants,
 * written to out7 [7] (device, FP64) asynchronously on the context's stream, with the
 * reduction's per-workgroup partial sums in a fixed array of the library's own device memory
 * instead of the workspace.  The array holds 1024 partial sums of 4 doubles (32 KiB) on every
 * GPU the library runs on, until the process ends; each reduction workgroup loops over sites,
 * so every lattice lb_init accepts fits (a context needing more partial sums would be rejected
 * with LB_EINVAL).  Allocates nothing and does not synchronise.  All calls on one GPU share
 * its array, and every call rewrites the part it reads: calls that overlap in time on one GPU
 * (different streams) race.  Latched device-side conditions are left to lb_status_check. */
lb_status lb_invariants_noalloc(lb_ctx* c, double* out7);

/* Synchronise the stream and report any latched device-side condition. */
lb_status lb_status_check(lb_ctx* c);

/* Number of completed steps since lb_init (or since the last lb_state_load). */
int64_t lb_step_count(const lb_ctx* c);

/* Snapshot of the full dynamic state (populations, atom displacements and velocities,
 * step count): lb_state_bytes() bytes of caller device memory.  Asynchronous. */
size_t lb_state_bytes(const lb_ctx* c);
lb_status lb_state_save(lb_ctx* c, void* dst);
lb_status lb_state_load(lb_ctx* c, const void* src);

/* Kernel timing with HIP events recorded on the context's streams around each phase of
 * the next max_steps steps (creates 8 * max_steps events).  lb_timing_end synchronises and
 * writes out_ms[0] = summed duration of the lattice sweep kernels, out_ms[1] = summed
 * duration of the atom kernel chains (binning, coupling, cell sort + force field; the
 * integration, a few microseconds, is not bracketed), out_ms[2] = number of steps timed
 * (milliseconds; host pointer).  Chains on different streams overlap in time, so the sum
 * of out_ms[0] and out_ms[1] can exceed the wall time. */
lb_status lb_timing_begin(lb_ctx* c, int32_t max_steps);
lb_status lb_timing_end(lb_ctx* c, double out_ms[3]);

/* ---- Gradients (discrete adjoint of lb_couple_step) ------------------------------------
 * The friction coupling of Section 2.2 and the lattice step (Eqs. 1-3) are differentiated in
 * reverse mode, so that a loss L of the atoms' final positions (and velocities) yields
 * dL/dgamma, dL/dtau and dL/dF_ext, the derivative with respect to the external force density
 * at every site.  The forward pass is recomputed from checkpoints segment by segment
 * (checkpoint-and-recompute), so memory grows with k, not with the number of steps.
 *
 * Usage: save the state with lb_state_save into ckpts + s * lb_state_bytes(c) before each
 * segment s = 0, 1, ... of k steps (the last segment may be shorter), run all n_steps with
 * lb_couple_step, then call lb_backward.  Size of the adjoint workspace for segments of k
 * steps (0 if the context has no atoms or k < 1): */
size_t lb_adjoint_workspace_bytes(const lb_ctx* c, int32_t k);

/* ckpts     device, 256-aligned: ceil(n_steps / k) states of lb_state_bytes(c) each, the s-th
 *           taken k * s steps after the first; the context must now be n_steps after it
 *           (LB_ESTATE otherwise)
 * adj_ws    device, 256-aligned, adj_ws_bytes >= lb_adjoint_workspace_bytes(c, k) (LB_ENOMEM)
 * dL_dX     device [N][3]: dL/dX at the final step (unwrapped positions); required
 * dL_dv     device [N][3] dL/dv at the final step, or NULL for zero
 * dL_dgamma, dL_dtau   host, out (FP64 accumulation on the device)
 * dL_db     device [3][nz][ny][nx] out (FP32): dL/dF_ext summed over the steps, or NULL
 * dL_dX0, dL_dv0  device [N][3] out, or NULL: dL/dX and dL/dv at the first checkpoint's step
 *           (positions taken with the tether anchors held fixed)
 * The work is queued on the context's stream (and, for a two-stream context, on its atom
 * stream, forked from and joined with it); the call synchronises before returning.  The
 * context's state is restored to the one before the call.  Rounding of FP16/BF16 storage is
 * treated as the identity. */
lb_status lb_backward(lb_ctx* c, const void* ckpts, int32_t n_steps, int32_t k, void* adj_ws,
                      size_t adj_ws_bytes, const float* dL_dX, const float* dL_dv,
                      double* dL_dgamma, double* dL_dtau, float* dL_db, float* dL_dX0,
                      float* dL_dv0);

/* Release the context (host memory only; the workspace stays the caller's). */
lb_status lb_destroy(lb_ctx* c);

/* Message describing the last failure on this context (or of the last lb_init when c is
 * NULL).  Valid until the next call on the same context. */
const char* lb_last_error(const lb_ctx* c);

#ifdef __cplusplus
}
#endif

#endif /* LBMD_H */
