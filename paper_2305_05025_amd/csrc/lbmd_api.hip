// Host side of the C interface declared in include/lbmd.h: argument validation, the
// workspace plan, initial state, the per-step launch sequence and the synchronising calls.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "lbmd_internal.h"

namespace lbmd {

static size_t round_up(size_t n, size_t a) { return (n + a - 1) / a * a; }

static size_t elem_bytes(int storage) { return storage == LB_STORE_F32 ? 4 : 2; }

bool geometry(const lb_params* p, Geometry* g) {
  g->q = p->velocity_set == 27 ? 27 : 19;
  g->nx = p->L[0];
  g->ny = p->L[1];
  g->nz = p->L[2];
  g->S = (long)p->L[0] * p->L[1] * p->L[2];
  g->plane = (long)round_up((size_t)g->S, 64) + kPlanePad;
  g->nblocks = (int)((g->S + kSweepBlock - 1) / kSweepBlock);
  g->ntiles = (int)((g->S + 63) / 64);
  g->nb[0] = (g->nx + kBrickX - 1) / kBrickX;
  g->nb[1] = (g->ny + kBrickY - 1) / kBrickY;
  g->nb[2] = (g->nz + kBrickZ - 1) / kBrickZ;
  g->nbricks = (long)g->nb[0] * g->nb[1] * g->nb[2];
  g->elem = elem_bytes(p->storage);
  g->div_nx = make_fastdiv((uint32_t)g->nx);
  g->div_ny = make_fastdiv((uint32_t)g->ny);
  g->narrow = (uint64_t)g->S * g->elem <= (1ull << 32) && std::getenv("LBMD_WIDE_OFFSETS") == nullptr;
  // the sweep's population bytes per step (every value read and written once) per atom
  const double sweep_bytes = (double)g->S * 2.0 * g->q * (double)g->elem;
  g->late_forces = std::getenv("LBMD_LATE_FORCES") != nullptr ||
                   (g->S >= (1L << 23) && sweep_bytes >= 7168.0 * (double)p->n_atoms);
  g->fused = (p->flags & LB_FLAG_FUSED_COUPLING) != 0 && p->n_atoms > 0;
  g->overlap = p->n_atoms > 0 && !(p->flags & LB_FLAG_SINGLE_STREAM) &&
               (g->S > (long)LB_ONE_STREAM_MAX_SITES || std::getenv("LBMD_OVERLAP_SMALL") != nullptr);
  g->ncell = 0;
  for (int k = 0; k < 3; ++k) {
    g->nc[k] = 0;
    g->inv_cw[k] = 0.f;
  }
  if (p->n_atoms > 0 && (p->lj_eps != 0.0f || p->coul_k != 0.0f)) {
    g->ncell = 1;
    for (int k = 0; k < 3; ++k) {
      // cells at least r_c (plus a 0.1% margin against rounding of wrapped positions) wide
      g->nc[k] = (int)std::floor((double)p->L[k] / ((double)p->lj_rc * 1.001));
      if (g->nc[k] < 3) return false;
      g->inv_cw[k] = (float)((double)g->nc[k] / (double)p->L[k]);
      g->ncell *= g->nc[k];
    }
  }
  return true;
}

size_t plan_bin(const lb_params* p, const Geometry& g, bool one_parity, Layout* l) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up(bytes, 256);
    return o;
  };
  // [step parity] buffers: two, or one shared by both parities
  auto take2 = [&](size_t (&o)[2], size_t bytes) {
    o[0] = take(bytes);
    o[1] = one_parity ? o[0] : take(bytes);
  };
  const size_t N = (size_t)p->n_atoms;
  take2(l->fcoup, N ? 3 * (size_t)g.plane * 4 : 0);
  take2(l->tile_flag, N ? (size_t)g.ntiles * 4 : 0);
  take2(l->base_count, N ? (size_t)g.plane * 4 : 0);
  take2(l->base_list, N ? (size_t)g.plane * kBaseCap * 4 : 0);
  l->uc = take(N ? 3 * (size_t)g.plane * 4 : 0);
  l->atom_frac = take(N * 16);
  l->occ_cells = take(std::min((size_t)g.ncell, N) * 4);
  take2(l->occ_tiles, N ? (size_t)g.ntiles * 4 : 0);
  take2(l->node_list, std::min(8 * N, (size_t)g.S) * 4);
  take2(l->occ_count, N ? 16 : 0);
  l->fc = take(3 * N * 4);
  l->cell_count = take((size_t)g.ncell * 4);
  l->cell_rec = take((size_t)g.ncell * kCellCap * 16);
  l->U = take(3 * N * 4);
  return off;
}

Layout plan(const lb_params* p, const Geometry& g) {
  Layout l;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += round_up(bytes, 256);
    return o;
  };
  const size_t N = (size_t)p->n_atoms;
  const size_t popb = (size_t)g.q * g.plane * g.elem;
  l.pop[0] = take(popb);
  l.pop[1] = take(popb);
  l.bin_bytes = plan_bin(p, g, false, &l);
  l.bin_base = take(l.bin_bytes);
  l.node_flag = take(N ? (size_t)g.plane : 0);
  for (int k = 0; k < 2; ++k) {
    l.brick_count[k] = take(g.fused ? (size_t)g.nbricks * 4 : 0);
    l.brick_list[k] = take(g.fused ? (size_t)g.nbricks * kBrickCap * 4 : 0);
    l.hot_bricks[k] = take(g.fused ? (size_t)g.nbricks * 4 : 0);
  }
  l.fext_tab = take((size_t)g.ny * 4);
  l.fext_field = take(p->bf_kind == LB_BF_FIELD ? 3 * (size_t)g.plane * 4 : 0);
  l.x0 = take(3 * N * 4);
  // displacement and velocity: float-float pairs, all hi parts then all lo parts
  l.disp[0] = take(2 * 3 * N * 4);
  l.disp[1] = take(2 * 3 * N * 4);
  l.vel = take(2 * 3 * N * 4);
  l.ff = take(3 * N * 4);
  l.charge = take(N * 4);
  l.bond_off = take((N + 1) * 4);
  l.bond_nbr = take(2 * (size_t)p->n_bonds * 4);
  l.red_partial = take((size_t)kRedBlocks * 4 * 8);
  l.red_out = take(8 * 8);
  l.err = take(4 * 4);
  l.total = off;
  return l;
}

static bool finite(float x) { return std::isfinite(x); }

// Returns an empty string when the parameters are valid.
static std::string validate(const lb_params* p) {
  char buf[256];
  if (!p) return "params is NULL";
  for (int k = 0; k < 3; ++k)
    if (p->L[k] < 2) {
      std::snprintf(buf, sizeof buf, "L[%d] = %d: every lattice extent must be >= 2", k, p->L[k]);
      return buf;
    }
  const double S = (double)p->L[0] * p->L[1] * p->L[2];
  if (S > 2147483647.0) return "lattice has more than 2^31 - 1 sites";
  if (!finite(p->tau) || !(p->tau > 0.5f)) return "tau must be finite and > 0.5 (nu = (tau - 1/2)/3 > 0)";
  if (p->flags & ~(LB_FLAG_CHECK_FINITE | LB_FLAG_SINGLE_STREAM | LB_FLAG_FUSED_COUPLING | LB_FLAG_STEP_GRAPHS))
    return "flags holds an unknown bit";
  if (!finite(p->kT) || p->kT < 0.0f) return "kT must be finite and >= 0";
  if (!finite(p->trt_magic) || p->trt_magic < 0.0f) return "trt_magic must be finite and >= 0";
  if (p->velocity_set != 0 && p->velocity_set != 19 && p->velocity_set != 27)
    return "velocity_set must be 19 or 27 (0 means 19)";
  if (!finite(p->rho0) || !(p->rho0 > 0.0f)) return "rho0 must be finite and > 0";
  if (p->storage < LB_STORE_F32 || p->storage > LB_STORE_BF16) return "unknown storage format";
  if (p->bf_kind < LB_BF_NONE || p->bf_kind > LB_BF_FIELD) return "unknown body-force kind";
  if (!finite(p->bf_amp)) return "bf_amp must be finite";
  if (p->n_atoms < 0 || p->n_atoms > (1 << 27)) return "n_atoms must be in [0, 2^27]";
  if (p->n_bonds < 0) return "n_bonds must be >= 0";
  if (p->n_atoms > 0) {
    if (!finite(p->mass) || !(p->mass > 0.0f)) return "mass must be finite and > 0";
    if (!finite(p->gamma) || p->gamma < 0.0f) return "gamma must be finite and >= 0";
    if (!finite(p->k_tether)) return "k_tether must be finite";
    if (!finite(p->k_bond) || !finite(p->r0_bond)) return "bond parameters must be finite";
    if (!finite(p->lj_eps) || p->lj_eps < 0.0f) return "lj_eps must be finite and >= 0";
    if (!finite(p->coul_k)) return "coul_k must be finite";
    if (p->lj_eps != 0.0f && (!finite(p->lj_sigma) || !(p->lj_sigma > 0.0f))) return "lj_sigma must be > 0";
    if (p->lj_eps != 0.0f || p->coul_k != 0.0f) {
      // cell-relative fixed-point positions (8.24) need cells narrower than ~60 lattice units
      if (!finite(p->lj_rc) || !(p->lj_rc > 0.0f) || p->lj_rc > 40.0f) return "lj_rc must be in (0, 40]";
      for (int k = 0; k < 3; ++k)
        if (std::floor((double)p->L[k] / ((double)p->lj_rc * 1.001)) < 3) {
          std::snprintf(buf, sizeof buf,
                        "L[%d] = %d is shorter than 3 Lennard-Jones cut-offs (%g): the cell list "
                        "needs 3 cells per axis",
                        k, p->L[k], (double)p->lj_rc);
          return buf;
        }
    }
  } else if (p->n_bonds > 0) {
    return "bonds given without atoms";
  }
  return "";
}

}  // namespace lbmd

using namespace lbmd;

static thread_local std::string g_init_error;

static lb_status fail(lb_ctx* c, lb_status s, const std::string& msg) {
  if (c)
    c->err = msg;
  else
    g_init_error = msg;
  return s;
}

static lb_status hip_fail(lb_ctx* c, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return fail(c, LB_EDEVICE, m);
}

extern "C" {

lb_status lb_velocity_set_q(int32_t q, int8_t* c, double* w) {
  if (q != 19 && q != 27) return fail(nullptr, LB_EINVAL, "q must be 19 or 27");
  static const double w19[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
  static const double w27[4] = {8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0};
  for (int i = 0; i < q; ++i) {
    if (c) {
      c[3 * i] = (int8_t)CX[i];
      c[3 * i + 1] = (int8_t)CY[i];
      c[3 * i + 2] = (int8_t)CZ[i];
    }
    const int n2 = CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i];
    if (w) w[i] = q == 27 ? w27[n2] : w19[n2];
  }
  return LB_OK;
}

void lb_velocity_set(int8_t c[19][3], double w[19]) {
  static const double wq[3] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 36.0};
  for (int i = 0; i < 19; ++i) {
    if (c) {
      c[i][0] = (int8_t)CX[i];
      c[i][1] = (int8_t)CY[i];
      c[i][2] = (int8_t)CZ[i];
    }
    if (w) w[i] = wq[CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]];
  }
}

size_t lb_workspace_bytes(const lb_params* p) {
  if (!validate(p).empty()) return 0;
  Geometry g;
  if (!geometry(p, &g)) return 0;
  return plan(p, g).total;
}

lb_status lb_init(const lb_params* p, void* workspace, size_t workspace_bytes, const float* x0,
                  const float* v0, const int32_t* bonds, const float* body_force,
                  void* hip_stream, lb_ctx** out) {
  if (!out) return fail(nullptr, LB_EINVAL, "out is NULL");
  *out = nullptr;
  const std::string why = validate(p);
  if (!why.empty()) return fail(nullptr, LB_EINVAL, why);
  Geometry g;
  if (!geometry(p, &g)) return fail(nullptr, LB_EINVAL, "cell-list geometry is invalid");
  const Layout lay = plan(p, g);
  if (!workspace) return fail(nullptr, LB_EINVAL, "workspace is NULL");
  if ((uintptr_t)workspace % 256 != 0) return fail(nullptr, LB_ENOMEM, "workspace must be 256-byte aligned");
  if (workspace_bytes < lay.total) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "workspace holds %zu bytes, %zu needed", workspace_bytes, lay.total);
    return fail(nullptr, LB_ENOMEM, buf);
  }
  const int N = p->n_atoms;
  if (N > 0 && (!x0 || !v0)) return fail(nullptr, LB_EINVAL, "x0 and v0 are required when n_atoms > 0");
  if (p->n_bonds > 0 && !bonds) return fail(nullptr, LB_EINVAL, "bonds is NULL but n_bonds > 0");
  if (p->bf_kind == LB_BF_FIELD && !body_force) return fail(nullptr, LB_EINVAL, "body_force field is NULL");
  hipStream_t st = (hipStream_t)hip_stream;

  // inputs read back once for validation and for the per-atom bond lists
  std::vector<float> hx(3 * (size_t)N), hv(3 * (size_t)N);
  std::vector<int32_t> hb(2 * (size_t)p->n_bonds);
  hipError_t e;
  if (N > 0) {
    if ((e = hipMemcpyAsync(hx.data(), x0, hx.size() * 4, hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(nullptr, e, "reading x0");
    if ((e = hipMemcpyAsync(hv.data(), v0, hv.size() * 4, hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(nullptr, e, "reading v0");
  }
  if (p->n_bonds > 0 &&
      (e = hipMemcpyAsync(hb.data(), bonds, hb.size() * 4, hipMemcpyDeviceToHost, st)) != hipSuccess)
    return hip_fail(nullptr, e, "reading bonds");
  if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(nullptr, e, "synchronising");
  for (size_t k = 0; k < hx.size(); ++k) {
    if (!std::isfinite(hx[k]) || std::fabs(hx[k]) > 1.0e6f)
      return fail(nullptr, LB_EINVAL, "x0 holds a non-finite or out-of-range (|x| > 1e6) coordinate");
    if (!std::isfinite(hv[k])) return fail(nullptr, LB_EINVAL, "v0 holds a non-finite value");
  }
  std::vector<int32_t> off(N + 1, 0), nbr(2 * (size_t)p->n_bonds);
  for (int b = 0; b < p->n_bonds; ++b) {
    const int i = hb[2 * b], j = hb[2 * b + 1];
    if (i < 0 || i >= N || j < 0 || j >= N || i == j) {
      char buf[128];
      std::snprintf(buf, sizeof buf, "bond %d = (%d, %d) is not a pair of distinct atoms", b, i, j);
      return fail(nullptr, LB_EINVAL, buf);
    }
    off[i + 1]++;
    off[j + 1]++;
  }
  for (int i = 0; i < N; ++i) off[i + 1] += off[i];
  {
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int b = 0; b < p->n_bonds; ++b) {
      const int i = hb[2 * b], j = hb[2 * b + 1];
      nbr[fill[i]++] = j;
      nbr[fill[j]++] = i;
    }
  }
  std::vector<float> tab(g.ny, 0.0f);
  for (int y = 0; y < g.ny; ++y) {
    if (p->bf_kind == LB_BF_KOLMOGOROV) {
      tab[y] = (float)((double)p->bf_amp * std::sin(2.0 * M_PI * (double)y / (double)g.ny));
    } else if (p->bf_kind == LB_BF_SIGN_SHEAR) {
      const double a = (double)y + 0.5 - 0.5 * (double)g.ny;
      tab[y] = (float)((double)p->bf_amp * (a > 0 ? 1.0 : (a < 0 ? -1.0 : 0.0)));
    }
  }

  int device = 0;
  if ((e = hipGetDevice(&device)) != hipSuccess) return hip_fail(nullptr, e, "querying the device");
  if ((e = setup_invariants_scratch(device)) != hipSuccess)
    return hip_fail(nullptr, e, "looking up the reduction scratch on this device");
  lb_ctx* c = new (std::nothrow) lb_ctx();
  if (!c) return fail(nullptr, LB_ENOMEM, "host allocation failed");
  c->p = *p;
  c->device = device;
  c->geo = g;
  c->lay = lay;
  c->stream = st;
  c->ws = (char*)workspace;
  c->bin = c->ws + lay.bin_base;
  c->popbuf[0] = c->ws + lay.pop[0];
  c->popbuf[1] = c->ws + lay.pop[1];
  c->cur = 0;
  c->dcur = 0;
  c->step = 0;
  c->omega = 1.0f / p->tau;
  c->omega_m = p->trt_magic > 0.0f
                   ? (float)(1.0 / (0.5 + (double)p->trt_magic / ((double)p->tau - 0.5)))
                   : c->omega;

  char* ws = c->ws;
  // zero everything the step relies on being zero (the binning region as a whole)
  const size_t popb = (size_t)g.q * g.plane * g.elem;
  struct Z { size_t off, bytes; } zs[] = {
      {lay.pop[0], popb}, {lay.pop[1], popb}, {lay.bin_base, lay.bin_bytes},
      {lay.node_flag, N ? (size_t)g.plane : 0},
      {lay.disp[0], 24 * (size_t)N}, {lay.disp[1], 24 * (size_t)N},
      {lay.vel, 24 * (size_t)N}, {lay.err, 16},
      {lay.fext_field, p->bf_kind == LB_BF_FIELD ? 3 * (size_t)g.plane * 4 : 0}};
  for (const Z& z : zs)
    if (z.bytes && (e = launch_zero(ws + z.off, round_up(z.bytes, 4), st)) != hipSuccess) {
      delete c;
      return hip_fail(nullptr, e, "clearing the workspace");
    }
  auto h2d = [&](size_t o, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(ws + o, src, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  auto d2d = [&](size_t o, const void* src, size_t bytes) {
    return bytes ? hipMemcpyAsync(ws + o, src, bytes, hipMemcpyDeviceToDevice, st) : hipSuccess;
  };
  if ((e = d2d(lay.x0, x0, 12 * (size_t)N)) != hipSuccess ||
      (e = d2d(lay.vel, v0, 12 * (size_t)N)) != hipSuccess ||
      (e = h2d(lay.fext_tab, tab.data(), 4 * (size_t)g.ny)) != hipSuccess ||
      (e = h2d(lay.bond_off, off.data(), 4 * off.size())) != hipSuccess ||
      (e = h2d(lay.bond_nbr, nbr.data(), 4 * nbr.size())) != hipSuccess) {
    delete c;
    return hip_fail(nullptr, e, "copying inputs");
  }
  if (p->bf_kind == LB_BF_FIELD)
    for (int k = 0; k < 3; ++k)
      if ((e = d2d(lay.fext_field + 4 * (size_t)k * g.plane, body_force + (size_t)k * g.S,
                   4 * (size_t)g.S)) != hipSuccess) {
        delete c;
        return hip_fail(nullptr, e, "copying the body-force field");
      }
  // the host vectors must outlive the copies
  if ((e = hipStreamSynchronize(st)) != hipSuccess) {
    delete c;
    return hip_fail(nullptr, e, "synchronising after set-up");
  }
  c->astream = st;
  if (g.overlap) {
    // atom work that overlaps the sweep runs on one more stream (default priority).  The
    // events inside a step are waited on only by this device's kernels, so they release at
    // device scope (no system-scope fence; about 4 us less per step); the fork and join with
    // the caller's stream keep the default.
    const unsigned dev_ev = hipEventDisableTiming | hipEventDisableSystemFence;
    if ((e = hipStreamCreateWithFlags(&c->astream, hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_bin, dev_ev)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_spread, dev_ev)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_couple, dev_ev)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming)) != hipSuccess) {
      lb_destroy(c);
      return hip_fail(nullptr, e, "creating the atom stream");
    }
    if (g.fused)
      for (int k = 0; k < 2 && e == hipSuccess; ++k)
        if ((k == 0 && (e = hipStreamCreateWithFlags(&c->hstream, hipStreamNonBlocking)) != hipSuccess) ||
            (e = hipEventCreateWithFlags(&c->ev_hot[k], dev_ev)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&c->ev_cold[k], dev_ev)) != hipSuccess) {
          lb_destroy(c);
          return hip_fail(nullptr, e, "creating the hot-brick stream");
        }
  }
  if ((p->flags & LB_FLAG_STEP_GRAPHS) &&
      (e = hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking)) != hipSuccess) {
    lb_destroy(c);
    return hip_fail(nullptr, e, "creating the capture stream");
  }
  *out = c;
  return LB_OK;
}

// The fused step.  Three streams: the caller's ("cold"), "hot" and "atoms".  Step n:
//   hot:    wait ev_bin(n) and ev_cold(n - 1); hot-brick sweep (coupling of step n, update of the
//           hot bricks' sites) -> ev_hot(n)
//   cold:   wait ev_bin(n) and ev_hot(n - 1); sweep of every other site -> ev_cold(n)
//   atoms:  (binning, cell sort and force field at X^n done) wait ev_hot(n); integration with
//           the friction of step n; then, for step n + 1: binning -> ev_bin(n + 1), cell sort,
//           force field at X^{n+1}
// The two sweeps of a step read the populations of step n and write disjoint sites of step
// n + 1, so they run side by side; the hot sweep of step n + 1 reads the halo of its bricks,
// written by both sweeps of step n, and the cold sweep of step n + 1 overwrites the buffer the
// hot sweep of step n reads.  The integration and the next step's binning, cell sort and force
// field overlap the cold sweep.  Per-step buffers written by the binning are double-buffered by
// step parity, so the sweeps of step n (which read step n's brick lists and counts) and the
// binning of step n + 1 never share one.  With LB_FLAG_SINGLE_STREAM every launch goes to the
// caller's stream: binning, cell sort, force field, hot bricks, the rest, integration.
static lb_status couple_step_fused(lb_ctx* c, int32_t n_steps) {
  const bool multi = c->astream != c->stream;
  hipStream_t hs = multi ? c->hstream : c->stream;
  hipError_t e;
  auto rec = [&](hipEvent_t* ev, int k, hipStream_t st) {
    if (ev) (void)hipEventRecord(ev[k], st);
  };
  auto slot = [&]() -> hipEvent_t* {
    return c->timed < c->timed_cap ? &c->ev[kTimedEvents * (size_t)c->timed] : nullptr;
  };
  // binning of the current step, its cell sort and the force field at its positions, on the
  // atom stream
  auto atom_prologue = [&](hipEvent_t* ev) -> lb_status {
    rec(ev, 4, c->astream);
    if ((e = launch_brick_binning(c)) != hipSuccess) return hip_fail(c, e, "binning launch");
    rec(ev, 5, c->astream);
    if (multi && (e = hipEventRecord(c->ev_bin, c->astream)) != hipSuccess) return hip_fail(c, e, "binning event");
    if (c->geo.ncell > 0 && (e = launch_cell_sort(c)) != hipSuccess) return hip_fail(c, e, "cell sort launch");
    rec(ev, 6, c->astream);
    if ((e = launch_forces(c)) != hipSuccess) return hip_fail(c, e, "force launch");
    rec(ev, 7, c->astream);
    return LB_OK;
  };
  if (multi) {
    if ((e = hipEventRecord(c->ev_fork, c->stream)) != hipSuccess ||
        (e = hipStreamWaitEvent(c->astream, c->ev_fork, 0)) != hipSuccess ||
        (e = hipStreamWaitEvent(hs, c->ev_fork, 0)) != hipSuccess)
      return hip_fail(c, e, "stream fork");
  }
  lb_status st;
  hipEvent_t* ev = slot();
  if (ev) c->timed++;
  if ((st = atom_prologue(ev)) != LB_OK) return st;
  for (int n = 0; n < n_steps; ++n) {
    void* fin = c->popbuf[c->cur];
    void* fout = c->popbuf[c->cur ^ 1];
    const int par = (int)(c->step & 1);
    if (multi && ((e = hipStreamWaitEvent(hs, c->ev_bin, 0)) != hipSuccess ||
                  (n > 0 && (e = hipStreamWaitEvent(hs, c->ev_cold[par ^ 1], 0)) != hipSuccess)))
      return hip_fail(c, e, "hot sweep wait");
    rec(ev, 0, hs);
    if ((e = launch_hot_sweep(c, fin, fout, hs)) != hipSuccess) return hip_fail(c, e, "hot sweep launch");
    rec(ev, 1, hs);
    if (multi && (e = hipEventRecord(c->ev_hot[par], hs)) != hipSuccess) return hip_fail(c, e, "hot sweep event");
    // the cold sweep skips the bricks this step's binning marked hot
    if (multi && ((e = hipStreamWaitEvent(c->stream, c->ev_bin, 0)) != hipSuccess ||
                  (n > 0 && (e = hipStreamWaitEvent(c->stream, c->ev_hot[par ^ 1], 0)) != hipSuccess)))
      return hip_fail(c, e, "cold sweep wait");
    rec(ev, 2, c->stream);
    if ((e = launch_cold_sweep(c, fin, fout, c->stream)) != hipSuccess) return hip_fail(c, e, "sweep launch");
    rec(ev, 3, c->stream);
    if (multi && (e = hipEventRecord(c->ev_cold[par], c->stream)) != hipSuccess) return hip_fail(c, e, "cold sweep event");
    if (multi && (e = hipStreamWaitEvent(c->astream, c->ev_hot[par], 0)) != hipSuccess)
      return hip_fail(c, e, "coupling wait");
    if ((e = launch_integrate(c)) != hipSuccess) return hip_fail(c, e, "integration launch");
    c->cur ^= 1;
    c->dcur ^= 1;
    c->step++;
    if (n + 1 < n_steps) {
      ev = slot();
      if (ev) c->timed++;
      if ((st = atom_prologue(ev)) != LB_OK) return st;
    }
    if (c->p.flags & LB_FLAG_CHECK_FINITE) {
      if (multi && ((e = hipEventRecord(c->ev_join, c->astream)) != hipSuccess ||
                    (e = hipStreamWaitEvent(c->stream, c->ev_join, 0)) != hipSuccess))
        return hip_fail(c, e, "stream join");
      if ((st = lb_status_check(c)) != LB_OK) return st;
    }
  }
  if (multi) {
    // the atom stream has waited for the last hot sweep; the cold stream joins it
    if ((e = hipEventRecord(c->ev_join, c->astream)) != hipSuccess ||
        (e = hipStreamWaitEvent(c->stream, c->ev_join, 0)) != hipSuccess)
      return hip_fail(c, e, "stream join");
  }
  return LB_OK;
}

static lb_status couple_steps_eager(lb_ctx* c, int32_t n_steps);

// LB_FLAG_STEP_GRAPHS: the step's launches and events, captured once per step parity as a
// graph of two steps and replayed.  A captured call is self-contained: it forks the atom
// stream from an event recorded inside the capture, bins its first step inside it and joins
// the atom stream back at its end, so no operation in it waits on an event recorded outside
// the capture.  Two steps return the population and displacement buffers to where they
// started, so one graph serves every call that starts at that parity; kernel arguments hold
// no other per-step value without thermal noise (whose counter is the step).
static bool graph_eligible(const lb_ctx* c, int32_t n_steps) {
  return (c->p.flags & LB_FLAG_STEP_GRAPHS) && c->gstream && n_steps >= 2 && !(c->p.flags & LB_FLAG_CHECK_FINITE) &&
         !c->geo.fused && c->p.kT == 0.0f && c->timed_cap == 0 && !c->keep_coupling && !c->couple_u &&
         c->bin == c->ws + c->lay.bin_base && c->popbuf[0] == c->ws + c->lay.pop[0] &&
         c->popbuf[1] == c->ws + c->lay.pop[1];
}

static lb_status couple_steps_graph(lb_ctx* c, int32_t n_steps) {
  hipError_t e;
  const int par = (int)(c->step & 1);
  if (!c->gexec[par]) {
    // captured on the library's own stream (the caller's may be the legacy null stream, which
    // cannot be captured); the graph is launched on the caller's
    const int cur = c->cur, dcur = c->dcur;
    const int64_t step = c->step;
    const hipStream_t caller = c->stream, as = c->astream;
    if ((e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(c, e, "beginning the step capture");
    c->stream = c->gstream;
    if (as == caller) c->astream = c->gstream;   // single-stream schedule
    const lb_status st = couple_steps_eager(c, 2);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->gstream, &g);
    c->stream = caller;
    c->astream = as;
    // nothing ran: the two captured steps are launched below
    c->cur = cur;
    c->dcur = dcur;
    c->step = step;
    if (st != LB_OK || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return st != LB_OK ? st : hip_fail(c, e, "ending the step capture");
    }
    e = hipGraphInstantiate(&c->gexec[par], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      c->gexec[par] = nullptr;
      return hip_fail(c, e, "instantiating the step graph");
    }
  }
  int32_t done = 0;
  for (; done + 2 <= n_steps; done += 2) {
    if ((e = hipGraphLaunch(c->gexec[par], c->stream)) != hipSuccess) return hip_fail(c, e, "step graph launch");
    c->step += 2;
  }
  return done < n_steps ? couple_steps_eager(c, n_steps - done) : LB_OK;
}

lb_status lb_couple_step(lb_ctx* c, int32_t n_steps) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (n_steps < 0) return fail(c, LB_EINVAL, "n_steps must be >= 0");
  if (n_steps == 0) return LB_OK;
  if (c->p.n_atoms > 0 && c->geo.fused) return couple_step_fused(c, n_steps);
  if (graph_eligible(c, n_steps)) return couple_steps_graph(c, n_steps);
  return couple_steps_eager(c, n_steps);
}

// the unfused step, every launch and event enqueued by the host
static lb_status couple_steps_eager(lb_ctx* c, int32_t n_steps) {
  const bool atoms = c->p.n_atoms > 0;
  hipError_t e;
  // Two streams (the caller's "main" stream and "atoms").  Step n:
  //   main:   wait ev_bin(n); node u_c, couple (-> ev_couple); spread -> ev_spread; sweep
  //   atoms:  (after the binning of step n) cell sort, (wait ev_couple,) force field at X^n;
  //           wait ev_spread; integration; then, for step n + 1: prep, bin/mark, compaction
  //           -> ev_bin(n + 1)
  // The coupling and the sweep run back to back on one stream; the force field (which
  // needs only X^n) overlaps them, and the integration and the next step's binning overlap
  // the sweep.  The atom stream first waits for everything already queued on the caller's
  // stream, and the caller's stream finally waits for the atom stream, so the call behaves
  // as if it had been queued on the caller's stream alone.  With LB_FLAG_SINGLE_STREAM every
  // launch goes to the caller's stream in the same order.
  const bool multi = atoms && c->astream != c->stream;
  // With a long sweep the force field waits for the coupling kernels (ev_couple), so that u_c
  // and the interpolation run without it beside them; it still takes its workgroup slots
  // before the sweep is launched.  Otherwise it starts right after the cell sort: on small
  // lattices the step is bound by the host's enqueue time and the extra event costs more than
  // it saves, and with a short sweep (16-bit storage) the atom loop is the longer cycle and
  // must not start later.  Both orders give identical bits.
  const bool late_forces = multi && c->geo.late_forces;
  auto rec = [&](hipEvent_t* ev, int k, hipStream_t st) {
    if (ev) (void)hipEventRecord(ev[k], st);
  };
  auto slot = [&]() -> hipEvent_t* {
    return c->timed < c->timed_cap ? &c->ev[kTimedEvents * (size_t)c->timed] : nullptr;
  };
  // per-step buffers read by the binning: see the ordering above
  auto binning = [&](hipEvent_t* ev) -> lb_status {
    rec(ev, 4, c->astream);
    if ((e = launch_prep(c)) != hipSuccess) return hip_fail(c, e, "prep launch");
    if ((e = launch_bin_mark(c)) != hipSuccess) return hip_fail(c, e, "binning launch");
    if ((e = launch_compact(c)) != hipSuccess) return hip_fail(c, e, "compaction launch");
    rec(ev, 5, c->astream);
    if (multi && (e = hipEventRecord(c->ev_bin, c->astream)) != hipSuccess) return hip_fail(c, e, "binning event");
    return LB_OK;
  };
  if (multi) {
    if ((e = hipEventRecord(c->ev_fork, c->stream)) != hipSuccess ||
        (e = hipStreamWaitEvent(c->astream, c->ev_fork, 0)) != hipSuccess)
      return hip_fail(c, e, "stream fork");
  }
  lb_status st;
  for (int n = 0; n < n_steps; ++n) {
    hipEvent_t* ev = slot();
    if (ev) c->timed++;
    void* fin = c->popbuf[c->cur];
    void* fout = c->popbuf[c->cur ^ 1];
    if (atoms) {
      if ((n == 0 || !multi) && (st = binning(ev)) != LB_OK) return st;
      if (multi && (e = hipStreamWaitEvent(c->stream, c->ev_bin, 0)) != hipSuccess)
        return hip_fail(c, e, "binning wait");
      // the cell sort and the force field (which needs only X^n) follow the binning on the
      // atom stream; see late_forces for where the force field starts.  (An event's record is
      // queued before the wait that refers to it.)
      if (c->geo.ncell > 0 && (e = launch_cell_sort(c)) != hipSuccess) return hip_fail(c, e, "cell sort launch");
      auto forces = [&]() -> lb_status {
        rec(ev, 6, c->astream);
        if ((e = launch_forces(c)) != hipSuccess) return hip_fail(c, e, "force launch");
        rec(ev, 7, c->astream);
        return LB_OK;
      };
      if (!late_forces && (st = forces()) != LB_OK) return st;
      rec(ev, 0, c->stream);
      if ((e = launch_node_u(c)) != hipSuccess) return hip_fail(c, e, "node velocity launch");
      if ((e = launch_couple(c)) != hipSuccess) return hip_fail(c, e, "coupling launch");
      if (late_forces) {
        if ((e = hipEventRecord(c->ev_couple, c->stream)) != hipSuccess ||
            (e = hipStreamWaitEvent(c->astream, c->ev_couple, 0)) != hipSuccess)
          return hip_fail(c, e, "coupling event");
        if ((st = forces()) != LB_OK) return st;
      }
      if ((e = launch_spread(c)) != hipSuccess) return hip_fail(c, e, "spread launch");
      rec(ev, 1, c->stream);
      if (multi && (e = hipEventRecord(c->ev_spread, c->stream)) != hipSuccess) return hip_fail(c, e, "spread event");
    }
    rec(ev, 2, c->stream);
    if ((e = launch_sweep(c, fin, fout, c->stream)) != hipSuccess) return hip_fail(c, e, "sweep launch");
    rec(ev, 3, c->stream);
    if (atoms) {
      if (multi && (e = hipStreamWaitEvent(c->astream, c->ev_spread, 0)) != hipSuccess)
        return hip_fail(c, e, "spread wait");
      if ((e = launch_integrate(c)) != hipSuccess) return hip_fail(c, e, "integration launch");
    }
    c->cur ^= 1;
    if (atoms) c->dcur ^= 1;
    c->step++;
    // the next binning rewrites the node flags and the atoms' stencil fractions, which this
    // step's spread reads: the atom stream has waited for ev_spread before the integration
    if (multi && n + 1 < n_steps && (st = binning(slot())) != LB_OK) return st;
    if (c->p.flags & LB_FLAG_CHECK_FINITE) {
      if (multi && ((e = hipEventRecord(c->ev_join, c->astream)) != hipSuccess ||
                    (e = hipStreamWaitEvent(c->stream, c->ev_join, 0)) != hipSuccess))
        return hip_fail(c, e, "stream join");
      if ((st = lb_status_check(c)) != LB_OK) return st;
    }
  }
  if (multi) {
    if ((e = hipEventRecord(c->ev_join, c->astream)) != hipSuccess ||
        (e = hipStreamWaitEvent(c->stream, c->ev_join, 0)) != hipSuccess)
      return hip_fail(c, e, "stream join");
  }
  return LB_OK;
}

lb_status lb_read_fields(lb_ctx* c, float* rho, float* u, float* x_unwrapped, float* v) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  hipError_t e;
  if ((rho || u) && (e = launch_read_fields(c, rho, u)) != hipSuccess) return hip_fail(c, e, "readback launch");
  if (c->p.n_atoms > 0 && (x_unwrapped || v) && (e = launch_read_atoms(c, x_unwrapped, v)) != hipSuccess)
    return hip_fail(c, e, "atom readback launch");
  return LB_OK;
}

lb_status lb_read_displacement(lb_ctx* c, float* d) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (!d) return fail(c, LB_EINVAL, "output is NULL");
  if (c->p.n_atoms == 0) return LB_OK;
  hipError_t e = hipMemcpyAsync(d, c->ws + c->lay.disp[c->dcur], 12 * (size_t)c->p.n_atoms,
                                hipMemcpyDeviceToDevice, c->stream);
  return e == hipSuccess ? LB_OK : hip_fail(c, e, "displacement copy");
}

lb_status lb_read_populations(lb_ctx* c, float* g) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (!g) return fail(c, LB_EINVAL, "output is NULL");
  hipError_t e = launch_read_populations(c, g);
  return e == hipSuccess ? LB_OK : hip_fail(c, e, "population readback launch");
}

lb_status lb_set_charges(lb_ctx* c, const float* q) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (c->p.n_atoms == 0) return LB_OK;
  if (!q) return fail(c, LB_EINVAL, "charges are NULL");
  hipError_t e = hipMemcpyAsync(c->ws + c->lay.charge, q, 4 * (size_t)c->p.n_atoms, hipMemcpyDeviceToDevice,
                                c->stream);
  return e == hipSuccess ? LB_OK : hip_fail(c, e, "charge copy");
}

lb_status lb_set_populations(lb_ctx* c, const float* g) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (!g) return fail(c, LB_EINVAL, "input is NULL");
  hipError_t e = launch_write_populations(c, g);
  return e == hipSuccess ? LB_OK : hip_fail(c, e, "population upload launch");
}

lb_status lb_status_check(lb_ctx* c) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  uint32_t err[4] = {0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(err, c->ws + c->lay.err, sizeof err, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "status read");
  if (err[0] & kErrOverflow)
    return fail(c, LB_EOVERFLOW, "a neighbour-list cell overflowed (atoms packed beyond any physical density)");
  if (err[0] & kErrNonFinite) return fail(c, LB_ENONFINITE, "a NaN or Inf appeared in the state");
  return LB_OK;
}

lb_status lb_invariants(lb_ctx* c, double out7[7]) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (!out7) return fail(c, LB_EINVAL, "out7 is NULL");
  hipError_t e = launch_invariants(c, (double*)(c->ws + c->lay.red_partial), (double*)(c->ws + c->lay.red_out));
  if (e != hipSuccess) return hip_fail(c, e, "invariants launch");
  double h[8];
  e = hipMemcpyAsync(h, c->ws + c->lay.red_out, sizeof h, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "invariants read");
  for (int k = 0; k < 7; ++k) out7[k] = h[k];
  return lb_status_check(c);
}

lb_status lb_invariants_noalloc(lb_ctx* c, double* out7) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (!out7) return fail(c, LB_EINVAL, "out7 is NULL");
  double* part = invariants_scratch(c->device);
  if (!part) return fail(c, LB_ESTATE, "the reduction scratch of this context's device is not set up");
  if (invariants_blocks(c) * 4 > kNoallocScratchDoubles) {
    char buf[160];
    std::snprintf(buf, sizeof buf, "the reduction needs %d partial sums, the fixed scratch holds %d",
                  invariants_blocks(c), kNoallocScratchDoubles / 4);
    return fail(c, LB_EINVAL, buf);
  }
  hipError_t e = launch_invariants(c, part, out7);
  return e == hipSuccess ? LB_OK : hip_fail(c, e, "invariants launch");
}

int64_t lb_step_count(const lb_ctx* c) { return c ? c->step : -1; }

// snapshot layout: [256-byte header: int64 step][populations][displacement hi, lo][velocity hi, lo]
static size_t state_pop_bytes(const lb_ctx* c) { return (size_t)c->geo.q * c->geo.plane * c->geo.elem; }

size_t lb_state_bytes(const lb_ctx* c) {
  if (!c) return 0;
  return 256 + round_up(state_pop_bytes(c), 256) + 2 * round_up(24 * (size_t)c->p.n_atoms, 256);
}

lb_status lb_state_save(lb_ctx* c, void* dst) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (!dst || (uintptr_t)dst % 256) return fail(c, LB_EINVAL, "dst must be a 256-byte aligned device buffer");
  char* d = (char*)dst;
  const size_t pb = round_up(state_pop_bytes(c), 256), ab = round_up(24 * (size_t)c->p.n_atoms, 256);
  hipError_t e = launch_store_i64(d, c->step, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(d + 256, c->popbuf[c->cur], state_pop_bytes(c), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && c->p.n_atoms > 0) {
    e = hipMemcpyAsync(d + 256 + pb, c->ws + c->lay.disp[c->dcur], 24 * (size_t)c->p.n_atoms,
                       hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(d + 256 + pb + ab, c->ws + c->lay.vel, 24 * (size_t)c->p.n_atoms,
                         hipMemcpyDeviceToDevice, c->stream);
  }
  return e == hipSuccess ? LB_OK : hip_fail(c, e, "state save");
}

lb_status lb_state_load(lb_ctx* c, const void* src) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (!src || (uintptr_t)src % 256) return fail(c, LB_EINVAL, "src must be a 256-byte aligned device buffer");
  const char* s = (const char*)src;
  const size_t pb = round_up(state_pop_bytes(c), 256), ab = round_up(24 * (size_t)c->p.n_atoms, 256);
  int64_t step = 0;
  hipError_t e = hipMemcpyAsync(&step, s, 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->popbuf[c->cur], s + 256, state_pop_bytes(c), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && c->p.n_atoms > 0) {
    e = hipMemcpyAsync(c->ws + c->lay.disp[c->dcur], s + 256 + pb, 24 * (size_t)c->p.n_atoms,
                       hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->ws + c->lay.vel, s + 256 + pb + ab, 24 * (size_t)c->p.n_atoms,
                         hipMemcpyDeviceToDevice, c->stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "state load");
  c->step = step;
  return LB_OK;
}

static void free_events(lb_ctx* c) {
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  c->timed_cap = c->timed = 0;
}

lb_status lb_timing_begin(lb_ctx* c, int32_t max_steps) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (max_steps < 0 || max_steps > (1 << 20)) return fail(c, LB_EINVAL, "max_steps must be in [0, 2^20]");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "synchronising");
  free_events(c);
  c->ev.resize(kTimedEvents * (size_t)max_steps);
  for (size_t k = 0; k < c->ev.size(); ++k)
    if ((e = hipEventCreate(&c->ev[k])) != hipSuccess) {
      c->ev.resize(k);
      free_events(c);
      return hip_fail(c, e, "creating timing events");
    }
  c->timed_cap = max_steps;
  c->timed = 0;
  return LB_OK;
}

lb_status lb_timing_end(lb_ctx* c, double out_ms[3]) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (!out_ms) return fail(c, LB_EINVAL, "out_ms is NULL");
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "synchronising");
  if (c->astream && c->astream != c->stream && (e = hipStreamSynchronize(c->astream)) != hipSuccess)
    return hip_fail(c, e, "synchronising");
  double sweep = 0.0, atoms = 0.0;
  const bool has_atoms = c->p.n_atoms > 0;
  // events per step: coupling 0-1, sweep 2-3, binning 4-5, force field 6-7
  for (int k = 0; k < c->timed; ++k) {
    float t[4] = {0.f, 0.f, 0.f, 0.f};
    hipEvent_t* ev = &c->ev[kTimedEvents * (size_t)k];
    for (int q = 0; q < (has_atoms ? 4 : 1); ++q) {
      const int a = q == 0 ? 2 : (q == 1 ? 0 : 2 * q);
      if ((e = hipEventElapsedTime(&t[q], ev[a], ev[a + 1])) != hipSuccess)
        return hip_fail(c, e, "reading timing events");
    }
    sweep += t[0];
    atoms += t[1] + t[2] + t[3];
  }
  out_ms[0] = sweep;
  out_ms[1] = atoms;
  out_ms[2] = c->timed;
  free_events(c);
  return LB_OK;
}

// ---- adjoint -------------------------------------------------------------------------------
namespace {

// final state, k state slots, k binning regions (one per step of a segment: the recomputed
// forward step q bins into region q and its backward step reads it there), adjoint fields
struct AdjLayout {
  size_t final_state, slots, sets, set_bytes, lam[2], phi, luc, lU, lf, lx[2], lv[2], lxa, dg_part,
      dom_part, acc, total;
  Layout set;  // the context's layout with the binning offsets of one step's region
};

AdjLayout plan_adjoint(const lb_ctx* c, int k) {
  AdjLayout l;
  l.set = c->lay;
  l.set_bytes = round_up(plan_bin(&c->p, c->geo, true, &l.set), 256);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = round_up(off + bytes, 256);
    return o;
  };
  const size_t sb = lb_state_bytes(c), N = (size_t)c->p.n_atoms, plane = (size_t)c->geo.plane;
  l.final_state = take(sb);
  l.slots = take(sb * (size_t)k);
  l.sets = take(l.set_bytes * (size_t)k);
  l.lam[0] = take((size_t)c->geo.q * plane * 4);
  l.lam[1] = take((size_t)c->geo.q * plane * 4);
  l.phi = take(3 * plane * 4);
  l.luc = take(3 * plane * 4);
  l.lU = take(12 * N);
  l.lf = take(16 * N);
  for (int q = 0; q < 2; ++q) {
    l.lx[q] = take(12 * N);
    l.lv[q] = take(12 * N);
  }
  l.lxa = take(12 * N);
  l.dg_part = take(8 * (size_t)adjoint_atom_blocks(c));
  l.dom_part = take(16 * (size_t)c->geo.nblocks);
  l.acc = take(24);
  l.total = off;
  return l;
}

// the atom part of a state record: displacement and velocity
size_t state_atom_offset(const lb_ctx* c) { return 256 + round_up(state_pop_bytes(c), 256); }

hipError_t copy_atoms(lb_ctx* c, char* dst_disp, char* dst_vel, const char* src_disp, const char* src_vel) {
  return launch_copy_pair(dst_disp, src_disp, dst_vel, src_vel, 24 * (size_t)c->p.n_atoms, c->stream);
}

}  // namespace

size_t lb_adjoint_workspace_bytes(const lb_ctx* c, int32_t k) {
  if (!c || k < 1 || c->p.n_atoms <= 0) return 0;
  return plan_adjoint(c, k).total;
}

lb_status lb_backward(lb_ctx* c, const void* ckpts, int32_t n_steps, int32_t k, void* adj_ws,
                      size_t adj_ws_bytes, const float* dL_dX, const float* dL_dv, double* dL_dgamma,
                      double* dL_dtau, float* dL_db, float* dL_dX0, float* dL_dv0) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  if (c->p.n_atoms <= 0) return fail(c, LB_EINVAL, "lb_backward needs atoms (the loss is a function of them)");
  if (n_steps < 1 || k < 1) return fail(c, LB_EINVAL, "n_steps and k must be >= 1");
  if (!ckpts || (uintptr_t)ckpts % 256) return fail(c, LB_EINVAL, "ckpts must be a 256-byte aligned device buffer");
  if (!adj_ws || (uintptr_t)adj_ws % 256) return fail(c, LB_EINVAL, "adj_ws must be a 256-byte aligned device buffer");
  if (!dL_dX) return fail(c, LB_EINVAL, "dL_dX is NULL");
  if (!dL_dgamma || !dL_dtau) return fail(c, LB_EINVAL, "dL_dgamma and dL_dtau are required (host)");
  const AdjLayout L = plan_adjoint(c, k);
  if (adj_ws_bytes < L.total) return fail(c, LB_ENOMEM, "adjoint workspace too small");
  const size_t sb = lb_state_bytes(c);
  const int n_seg = (n_steps + k - 1) / k;
  const char* ck = (const char*)ckpts;
  int64_t first = 0, last = 0;
  hipError_t e = hipMemcpyAsync(&first, ck, 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(&last, ck + (size_t)(n_seg - 1) * sb, 8, hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "reading the checkpoints");
  if (first + n_steps != c->step || last != first + (int64_t)(n_seg - 1) * k)
    return fail(c, LB_ESTATE, "checkpoints do not match: ckpts[s] must hold the state at step "
                              "(current step - n_steps) + s k");

  char* A = (char*)adj_ws;
  const size_t N3 = 3 * (size_t)c->p.n_atoms;
  const size_t aoff = state_atom_offset(c), abytes = round_up(24 * (size_t)c->p.n_atoms, 256);
  auto slot = [&](int q) { return A + L.slots + (size_t)q * sb; };
  auto set = [&](int q) { return A + L.sets + (size_t)q * L.set_bytes; };
  const hipStream_t as = c->astream;
  char* pb0 = c->popbuf[0];
  char* pb1 = c->popbuf[1];
  const Layout lay0 = c->lay;
  char* bin0 = c->bin;
  const bool fused0 = c->geo.fused;
  // step q of a segment bins into its own region (lay = L.set, bin = set(q))
  auto use_set = [&](int q) {
    c->lay = L.set;
    c->bin = set(q);
  };
  auto use_own = [&]() {
    c->lay = lay0;
    c->bin = bin0;
  };
  lb_status st = LB_OK;
  // the forward steps are recomputed by the unfused kernels (the same bits), each a one-step
  // call on the context's schedule, leaving the binning, coupling velocity, friction and
  // spread force of each step in its region; the other kernels of the backward pass run on the
  // caller's stream, except the force field's Hessian-vector product of each adjoint step,
  // which a two-stream context runs on its atom stream beside the lattice part
  c->astream = c->stream;
  c->geo.fused = false;
  if ((st = lb_state_save(c, A + L.final_state)) != LB_OK) goto restore;
  // the regions' spread force and base-node counts start at zero; each backward step clears
  // those of its step again (on the flagged tiles, where its forward step wrote them)
  for (int q = 0; q < k; ++q) {
    if ((e = launch_zero(set(q) + L.set.fcoup[0], 12 * (size_t)c->geo.plane, c->stream)) != hipSuccess ||
        (e = launch_zero(set(q) + L.set.base_count[0], 4 * (size_t)c->geo.plane, c->stream)) != hipSuccess) {
      st = hip_fail(c, e, "adjoint set-up");
      goto restore;
    }
  }
  if ((e = launch_zero(A + L.lam[0], (size_t)c->geo.q * c->geo.plane * 4, c->stream)) != hipSuccess ||
      (e = launch_zero(A + L.acc, 24, c->stream)) != hipSuccess ||
      (dL_db && (e = launch_zero(dL_db, 12 * (size_t)c->geo.S, c->stream)) != hipSuccess) ||
      (e = hipMemcpyAsync(A + L.lx[0], dL_dX, 4 * N3, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
      (e = dL_dv ? hipMemcpyAsync(A + L.lv[0], dL_dv, 4 * N3, hipMemcpyDeviceToDevice, c->stream)
                 : launch_zero(A + L.lv[0], 4 * N3, c->stream)) != hipSuccess) {
    st = hip_fail(c, e, "adjoint set-up");
    goto restore;
  }
  {
    int li = 0;
    for (int seg = n_seg - 1; seg >= 0; --seg) {
      const int t0 = seg * k, len = std::min(k, n_steps - t0);
      if ((e = hipMemcpyAsync(slot(0), ck + (size_t)seg * sb, sb, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess) {
        st = hip_fail(c, e, "checkpoint copy");
        goto restore;
      }
      // recompute the segment, each step's output going straight into the next slot (the
      // atoms' state of step q + 1 is still in the context when step q + 1 starts)
      for (int q = 0; q + 1 < len; ++q) {
        char* disp = c->ws + c->lay.disp[c->dcur];
        char* vel = c->ws + c->lay.vel;
        if (q == 0 && (e = copy_atoms(c, disp, vel, slot(q) + aoff, slot(q) + aoff + abytes)) != hipSuccess) {
          st = hip_fail(c, e, "recompute copy");
          goto restore;
        }
        c->popbuf[c->cur] = slot(q) + 256;
        c->popbuf[c->cur ^ 1] = slot(q + 1) + 256;
        c->step = first + t0 + q;
        use_set(q);
        c->couple_u = (float*)(set(q) + L.set.U);
        c->keep_coupling = true;
        c->astream = as;
        st = lb_couple_step(c, 1);
        c->astream = c->stream;
        c->keep_coupling = false;
        c->couple_u = nullptr;
        use_own();
        if (st != LB_OK) goto restore;
        if ((e = copy_atoms(c, slot(q + 1) + aoff, slot(q + 1) + aoff + abytes, c->ws + c->lay.disp[c->dcur],
                            c->ws + c->lay.vel)) != hipSuccess) {
          st = hip_fail(c, e, "recompute copy");
          goto restore;
        }
      }
      // the adjoint steps of the segment, last first
      for (int q = len - 1; q >= 0; --q) {
        if ((e = copy_atoms(c, c->ws + c->lay.disp[c->dcur], c->ws + c->lay.vel, slot(q) + aoff,
                            slot(q) + aoff + abytes)) != hipSuccess) {
          st = hip_fail(c, e, "adjoint copy");
          goto restore;
        }
        c->popbuf[c->cur] = slot(q) + 256;
        c->step = first + t0 + q;
        use_set(q);
        // the last step of the segment was not recomputed (its output is the next segment's
        // checkpoint): bin and couple it here
        if (q == len - 1) {
          c->couple_u = (float*)(set(q) + L.set.U);
          e = launch_prep(c);
          if (e == hipSuccess) e = launch_bin_mark(c);
          if (e == hipSuccess) e = launch_compact(c);
          if (e == hipSuccess && c->geo.ncell > 0) e = launch_cell_sort(c);
          if (e == hipSuccess) e = launch_node_u(c);
          if (e == hipSuccess) e = launch_couple(c);
          if (e == hipSuccess) e = launch_spread(c);
          c->couple_u = nullptr;
          if (e != hipSuccess) {
            st = hip_fail(c, e, "adjoint recompute launch");
            goto restore;
          }
        }
        AdjointBuffers b;
        b.lam_in = (const float*)(A + L.lam[li]);
        b.lam_out = (float*)(A + L.lam[li ^ 1]);
        b.phi = (float*)(A + L.phi);
        b.luc = (float*)(A + L.luc);
        b.db = dL_db;
        b.dom_part = (double*)(A + L.dom_part);
        b.dg_part = (double*)(A + L.dg_part);
        b.acc = (double*)(A + L.acc);
        b.U = (const float*)(set(q) + L.set.U);
        b.lU = (float*)(A + L.lU);
        b.lf = (float4*)(A + L.lf);
        b.lx_in = (const float*)(A + L.lx[li]);
        b.lv_in = (const float*)(A + L.lv[li]);
        b.lx_out = (float*)(A + L.lx[li ^ 1]);
        b.lv_out = (float*)(A + L.lv[li ^ 1]);
        b.lxa = (float*)(A + L.lxa);
        // the force field's Hessian-vector product beside the lattice part, on the atom
        // stream of a two-stream context (whose per-step events the recompute, run on one
        // stream here, leaves free)
        if (as != c->stream) {
          b.side = as;
          b.ev_fork = c->ev_couple;
          b.ev_join = c->ev_spread;
        }
        e = launch_adjoint_step(c, b);
        use_own();
        if (e != hipSuccess) {
          st = hip_fail(c, e, "adjoint step launch");
          goto restore;
        }
        li ^= 1;
      }
    }
    if ((dL_dX0 && (e = hipMemcpyAsync(dL_dX0, A + L.lx[li], 4 * N3, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess) ||
        (dL_dv0 && (e = hipMemcpyAsync(dL_dv0, A + L.lv[li], 4 * N3, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)) {
      st = hip_fail(c, e, "adjoint output");
      goto restore;
    }
    double acc[3];
    if ((e = hipMemcpyAsync(acc, A + L.acc, 24, hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess) {
      st = hip_fail(c, e, "adjoint result");
      goto restore;
    }
    *dL_dgamma = acc[0];
    // omega+ = 1/tau; omega- = omega+ (BGK) or 1/(1/2 + magic/(tau - 1/2)), whose derivative
    // is omega-^2 magic/(tau - 1/2)^2
    const double tau = c->p.tau, magic = c->p.trt_magic;
    double dtau = -acc[1] / (tau * tau);
    if (magic > 0.0) {
      const double om = 1.0 / (0.5 + magic / (tau - 0.5));
      dtau += acc[2] * om * om * magic / ((tau - 0.5) * (tau - 0.5));
    } else {
      dtau -= acc[2] / (tau * tau);
    }
    *dL_dtau = dtau;
  }
restore:
  c->couple_u = nullptr;
  c->keep_coupling = false;
  use_own();
  c->geo.fused = fused0;
  c->popbuf[0] = pb0;
  c->popbuf[1] = pb1;
  {
    const lb_status s2 = lb_state_load(c, A + L.final_state);
    c->astream = as;
    if (st == LB_OK) st = s2;
  }
  if (st == LB_OK) st = lb_status_check(c);
  return st;
}

lb_status lb_destroy(lb_ctx* c) {
  if (!c) return fail(nullptr, LB_EINVAL, "context is NULL");
  free_events(c);
  if (c->gexec[0] || c->gexec[1]) {
    (void)hipStreamSynchronize(c->stream);
    for (hipGraphExec_t g : c->gexec)
      if (g) (void)hipGraphExecDestroy(g);
  }
  for (hipStream_t s : {c->astream, c->hstream, c->gstream})
    if (s && s != c->stream) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  for (hipEvent_t e : {c->ev_fork, c->ev_bin, c->ev_couple, c->ev_spread, c->ev_join, c->ev_hot[0],
                       c->ev_hot[1], c->ev_cold[0], c->ev_cold[1]})
    if (e) (void)hipEventDestroy(e);
  delete c;
  return LB_OK;
}

const char* lb_last_error(const lb_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

}  // extern "C"
