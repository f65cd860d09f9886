// ktmi.hip -- host side and C ABI of libktmi (one RK2 step of the
// Kurganov-Tadmor scheme for (3+1)D viscous hydrodynamics in Milne
// coordinates, arXiv:1802.04449), plus the small per-cell kernels.  The
// stencil kernels are in ktmi_kernels.hpp; their instances and launchers come
// from the ktmi_stencil.hip objects.  The caller provides all device memory;
// nothing here allocates.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/ktmi.h"
#include "ktmi_kernels.hpp"
#include "ktmi_surface.hpp"

namespace ktmi {

// Initial primitive state: cutoff, then T~^{tau mu} = tau0 Tc^{tau mu}(e, u~, pi~)
// (ext: with P + Pi, and Pi, n zero below the cutoff).  pi~, Pi and n come
// staged in FP64 in the stage-1 block and go to the pi~ block in its storage type.
__global__ __launch_bounds__(kBlock) void k_init_primitive(Fields f, StepParams p, EosDev eos,
                                                            Geo g, int visc, int ext) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= p.ncell) return;
  double e = f.e[c];
  double u1 = f.u[0][c], u2 = f.u[1][c], u3 = f.u[2][c];
  double pv[10], Pi = ext ? f.pi1[10][c] : 0.0, nb = ext ? f.pi1[11][c] : 0.0;
#pragma unroll
  for (int m = 0; m < 10; ++m) pv[m] = visc ? f.pi1[m][c] : 0.0;
  if (!(e >= p.eps_cut)) {
    e = 0.0;
    u1 = u2 = u3 = 0.0;
#pragma unroll
    for (int m = 0; m < 10; ++m) pv[m] = 0.0;
    Pi = nb = 0.0;
  }
  if (ext) {
    stq_rt(f.pi[10], c, Pi, f.pf32);
    stq_rt(f.pi[11], c, nb, f.pf32);
  }
  double P, cs2;
  eos_p_cs2(eos, e, P, cs2);
  if (ext) P += Pi;
  const double ut = utau(u1, u2, u3);
  const double w = e + P;
  const double tf = g.cart ? 1.0 : g.tau;
  const double u4[4] = {ut, u1, u2, u3};
  f.e[c] = e;
  f.u[0][c] = u1;
  f.u[1][c] = u2;
  f.u[2][c] = u3;
#pragma unroll
  for (int m = 0; m < 10; ++m) stq_rt(f.pi[m], c, pv[m], f.pf32);
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) f.T[nu][c] = tf * (w * ut * u4[nu] - (nu == 0 ? P : 0.0) + pv[nu]);
}

// Folds the partials of stage1 and stage2T into the accumulated diagnostics.
// One workgroup of kRedBlock threads per slot; each folds the slot's partials
// in a fixed order (thread t takes tiles t, t + kRedBlock, ...; then the waves
// and the workgroup in order).
// acc: 0 geo_src, 1 max_cfl, 2 solves, 3 iter_sum, 4 iter_max, 5 fallbacks,
//      6 nonconv, 7 nans, 8 clamps, 9 eps_max, 10 sum_Ttt, 11 vacuum, 12 negative.
constexpr int kRedBlock = 1024;
__global__ __launch_bounds__(kRedBlock) void k_reduce(const EventDesc* __restrict__ evs) {
  __shared__ double sh[2][kRedBlock / 64];
  const int e = blockIdx.x / kNP, s = blockIdx.x % kNP;
  const EventDesc& E = evs[e];
  const int nblk = E.tg.ntiles;
  const gdouble* part = (const gdouble*)E.f.partial;
  const bool mx = is_max_slot(s);
  double x = 0.0, y = 0.0;  // stage1, stage2T
  // unrolled so that several rounds' loads are in flight; the folds keep their order
#pragma unroll 8
  for (int b = threadIdx.x; b < nblk; b += kRedBlock) {
    const double a = part[(size_t)s * nblk + b];
    const double c = part[(size_t)(kNP + s) * nblk + b];
    x = mx ? fmax(x, a) : x + a;
    y = mx ? fmax(y, c) : y + c;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double xo = __shfl_xor(x, off, 64), yo = __shfl_xor(y, off, 64);
    x = mx ? fmax(x, xo) : x + xo;
    y = mx ? fmax(y, yo) : y + yo;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wave] = x;
    sh[1][wave] = y;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  x = sh[0][0];
  y = sh[1][0];
  for (int w = 1; w < kRedBlock / 64; ++w) {
    x = mx ? fmax(x, sh[0][w]) : x + sh[0][w];
    y = mx ? fmax(y, sh[1][w]) : y + sh[1][w];
  }
  const double vol = E.p.dx * E.p.dy * E.p.de;
  double* acc = E.f.acc;
  switch (s) {
    case P_GEO: acc[0] += 0.5 * E.p.h * vol * (x + y); break;
    case P_CFL: acc[1] = fmax(acc[1], fmax(x, y)); break;
    case P_EMAX: acc[9] = y; break;
    case P_TSUM: acc[10] = y * vol; break;
    case P_VAC: acc[11] = y; break;
    case P_ITMAX: acc[4] = fmax(acc[4], fmax(x, y)); break;
    default: acc[s] += x + y; break;
  }
  if (s == 0) {  // advance the event's clock: tau += h, one more step, swap u~ buffers
    double* clk = E.clock;
    clk[0] = clk[0] + E.p.h;
    clk[1] = clk[1] + 1.0;
    clk[2] = 1.0 - clk[2];
  }
}

// Sets an event's clock at its initial state.
__global__ void k_set_clock(double* clk, double tau) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    clk[0] = tau;
    clk[1] = 0.0;
    clk[2] = 0.0;
  }
}

// pi~ as seen by readers: zero in vacuum cells; f32: stored in FP32.
__global__ __launch_bounds__(kBlock) void k_read_pi(const double* __restrict__ e,
                                                    const double* __restrict__ pi, double* dst,
                                                    int n, int f32) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c < n) dst[c] = e[c] == 0.0 ? 0.0 : ldq_rt(pi, c, f32);
}

// Copies the network parameters into the handle's workspace and appends W2 as BF16.
__global__ void k_mlp_pack(const float* __restrict__ src, float* __restrict__ dst) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < kMlpNParam) dst[k] = src[k];
  if (k < kMlpH * kMlpH)
    reinterpret_cast<uint16_t*>(dst + kMlpPad)[k] = (uint16_t)to_bf16(src[kOW2 + k]);
}

// Training samples from the current state: E = K^tau, M = |K|, with
// K = T~^{tau .}/tau - pi~^{tau .}, and the cell's e (the root of that K).
__global__ __launch_bounds__(kBlock) void k_harvest(Fields f, const double* __restrict__ clk,
                                                    int cart, int visc, int n,
                                                    double* __restrict__ E, double* __restrict__ M,
                                                    double* __restrict__ eps) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= n) return;
  const double tf = cart ? 1.0 : clk[0];
  const double e = f.e[c];
  const bool pv = visc && e != 0.0;
  const double K0 = f.T[0][c] / tf - (pv ? ldq_rt(f.pi[0], c, f.pf32) : 0.0);
  const double K1 = f.T[1][c] / tf - (pv ? ldq_rt(f.pi[1], c, f.pf32) : 0.0);
  const double K2 = f.T[2][c] / tf - (pv ? ldq_rt(f.pi[2], c, f.pf32) : 0.0);
  const double K3 = f.T[3][c] / tf - (pv ? ldq_rt(f.pi[3], c, f.pf32) : 0.0);
  E[c] = K0;
  M[c] = sqrt(K1 * K1 + K2 * K2 + K3 * K3);
  eps[c] = e;
}

__global__ void k_zero(double* p, int n) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c < n) p[c] = 0.0;
}

}  // namespace ktmi

// ===========================================================================
// Host side: handle, workspace layout and the C ABI.
// ===========================================================================
using namespace ktmi;

enum { K_INIT = 0, K_FIRST, K_STAGE1, K_STAGE2PI, K_STAGE2T, K_REDUCE, K_SURFACE, K_COUNT };
static const char* kKernelNames[K_COUNT] = {"init", "first_estimate", "stage1", "stage2_pi",
                                            "stage2_T", "reduce", "surface"};

struct ktmi_handle {
  ktmi_desc d;
  std::string err;
  unsigned long long* surf_blocks = nullptr;  // workspace scratch of the surface finder
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  bool bound = false, eos_set = false, ready = false;
  EosDev eos{};
  Fields f{};
  double* eos_store = nullptr;
  double cs2_vac = 1.0 / 3.0;  // cs2 of the EoS at e = 0
  double tau = 0.0;
  long step = 0;
  int nblk = 0;      // blocks of the flat (per-cell) kernels
  int tile = 0;      // index into kTiles
  TileGrid tg{};     // tile grid of the stencil kernels
  size_t fstride = 0;
  bool timing = false;
  struct Rec {
    int k;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  // device event table (one entry) and clock, both inside the workspace
  EventDesc ev{};           // host copy, kept alive for the asynchronous upload
  EventDesc* dev_ev = nullptr;
  double* clock = nullptr;
  bool ev_dirty = true;
  // graph of one step, replayed by ktmi_step when enabled
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  // learned root-solve guess: parameters copied into the workspace
  float* mlp_dev = nullptr;
  bool mlp_ok = false;
  // quiet-tile skipping (off by default); P of the EoS at e = 0 (must be 0 for it)
  bool quiet_on = false;
  double eos_p0 = 0.0;
  double p_at0 = 0.0;  // P as the device lookups give it at e = 0 (first row, or 0)
  int mlp_mode = KTMI_MLP_FP32;
};

static std::string g_create_err;

static int fail(ktmi_handle* h, int code, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    g_create_err = msg;
  return code;
}

static int hip_fail(ktmi_handle* h, hipError_t e, const char* what) {
  return fail(h, KTMI_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(h, call)                                   \
  do {                                                     \
    hipError_t _e = (call);                                \
    if (_e != hipSuccess) return hip_fail((h), _e, #call); \
  } while (0)

static bool desc_ok(const ktmi_desc* d, std::string* why) {
  if (!d) {
    *why = "null descriptor";
    return false;
  }
  if (d->nx < 1 || d->ny < 1 || d->ne < 1) {
    *why = "grid sizes must be >= 1";
    return false;
  }
  // the kernels address a field's elements by 32-bit byte offsets
  if ((double)d->nx * d->ny * d->ne > (double)((1u << 29) - 256)) {
    *why = "grid too large (more than 2^29 - 256 cells)";
    return false;
  }
  if (!(d->dx > 0) || !(d->dy > 0) || !(d->de > 0) || !(d->tau0 > 0) || !(d->h > 0)) {
    *why = "spacings, tau0 and h must be > 0";
    return false;
  }
  if (d->viscous && !(d->etas > 0)) {
    *why = "viscous mode needs etas > 0";
    return false;
  }
  if (d->viscous && !(d->taupi_coef > 0)) {
    *why = "viscous mode needs taupi_coef > 0";
    return false;
  }
  if (!std::isfinite(d->lambda1_hat)) {
    *why = "lambda1_hat must be finite";
    return false;
  }
  if (!(d->zetas >= 0.0) || !std::isfinite(d->zetas) || (d->baryon != 0 && d->baryon != 1)) {
    *why = "zetas must be finite and >= 0, baryon 0 or 1";
    return false;
  }
  if (d->zetas > 0.0 || d->baryon) {
    if (!d->viscous) {
      *why = "bulk pressure and baryon density need viscous mode";
      return false;
    }
    if (d->zetas > 0.0 && !(d->taubulk_coef > 0)) {
      *why = "bulk viscosity needs taubulk_coef > 0";
      return false;
    }
    if (d->precision != KTMI_FP64 || d->lambda1_hat != 0.0) {
      *why = "bulk pressure and baryon density run in FP64 without the lambda_1 term";
      return false;
    }
  }
  if (!(d->theta >= 1.0 && d->theta <= 2.0)) {
    *why = "theta must lie in [1, 2]";
    return false;
  }
  if (!(d->eps_cut > 0) || !(d->newton_tol > 0) || d->newton_maxit < 1) {
    *why = "eps_cut, newton_tol and newton_maxit must be positive";
    return false;
  }
  if (d->precision != KTMI_FP64 && d->precision != KTMI_MIXED) {
    *why = "precision must be KTMI_FP64 or KTMI_MIXED";
    return false;
  }
  if (d->guess != KTMI_GUESS_PREV && d->guess != KTMI_GUESS_COLD && d->guess != KTMI_GUESS_MLP) {
    *why = "unknown guess mode";
    return false;
  }
  if (d->tile < -1 || d->tile >= kNumTiles) {
    *why = "tile index out of range";
    return false;
  }
  if (!(d->cfl_limit > 0.0)) {
    *why = "cfl_limit must be > 0";
    return false;
  }
  return true;
}

static TileGrid tile_grid(const ktmi_desc* d, int t) {
  TileGrid g;
  g.ntx = (d->nx + kTiles[t].tx - 1) / kTiles[t].tx;
  g.nty = (d->ny + kTiles[t].ty - 1) / kTiles[t].ty;
  g.ntz = (d->ne + kTiles[t].tz - 1) / kTiles[t].tz;
  g.ntiles = g.ntx * g.nty * g.ntz;
  return g;
}

// Default tile: fewest padded thread slots, counting double for shapes whose eta
// extent is shorter than min(ne, 16) (their lanes stride across eta rows, so
// loads stop coalescing).  Ties keep list order.  The autotuner can override.
static int auto_tile(const ktmi_desc* d) {
  int best = 0;
  double best_score = 1e300;
  const int want_z = d->ne < 16 ? d->ne : 16;
  for (int t = 0; t < kNumTiles; ++t) {
    const double slots = (double)tile_grid(d, t).ntiles * kBlock;
    const double score = slots * (kTiles[t].tz >= want_z ? 1.0 : 2.0);
    if (score < best_score) {
      best_score = score;
      best = t;
    }
  }
  return best;
}

static int max_tiles(const ktmi_desc* d) {
  int m = 0;
  for (int t = 0; t < kNumTiles; ++t) m = std::max(m, tile_grid(d, t).ntiles);
  return m;
}

// Doubles reserved for the per-tile flags: 4 ints per tile of the largest grid
// (quiet flags by clock parity, the stage-2pi part, and stage 1's T~' = T~^n).
static size_t quiet_doubles(const ktmi_desc* d) {
  return ((size_t)4 * max_tiles(d) + 63) / 64 * 32;
}

static const int kNumFields = 39;  // e, u(3), up(3), pi(10), T(4), e1, u1(3), pi1(10), T1(4)

// Bulk pressure or baryon density in use: 4 more fields (Pi, n and their stage-1 values).
static bool has_ext(const ktmi_desc* d) { return d->zetas > 0.0 || d->baryon; }
static int num_fields(const ktmi_desc* d) { return kNumFields + (has_ext(d) ? 4 : 0); }

static size_t field_stride(const ktmi_desc* d) {
  const size_t n = (size_t)d->nx * d->ny * d->ne;
  return (n + 31) / 32 * 32;  // 256-byte aligned fields
}

static int num_blocks(const ktmi_desc* d) {
  const size_t n = (size_t)d->nx * d->ny * d->ne;
  return (int)((n + kBlock - 1) / kBlock);
}

static StepParams step_params(const ktmi_handle* h) {
  StepParams p;
  p.nx = h->d.nx;
  p.ny = h->d.ny;
  p.ne = h->d.ne;
  p.ncell = h->d.nx * h->d.ny * h->d.ne;
  p.dx = h->d.dx;
  p.dy = h->d.dy;
  p.de = h->d.de;
  p.inv_dx = 1.0 / h->d.dx;
  p.inv_dy = 1.0 / h->d.dy;
  p.inv_de = 1.0 / h->d.de;
  p.h = h->d.h;
  p.inv_h = 1.0 / h->d.h;
  p.etas = h->d.etas;
  const bool visc_ok = h->d.etas > 0 && h->d.taupi_coef > 0;
  p.inv_taupi_coef = visc_ok ? 1.0 / (h->d.taupi_coef * h->d.etas * kHbarc) : 0.0;
  p.eta_taupi = visc_ok ? 1.0 / h->d.taupi_coef : 0.0;
  p.lambda1_hat = h->d.lambda1_hat;
  const bool bulk_ok = h->d.zetas > 0 && h->d.taubulk_coef > 0;
  p.inv_taubulk_coef = bulk_ok ? 1.0 / (h->d.taubulk_coef * h->d.zetas * kHbarc) : 0.0;
  p.zeta_taubulk = bulk_ok ? 1.0 / h->d.taubulk_coef : 0.0;
  p.bulk = bulk_ok ? 1 : 0;
  p.baryon = h->d.baryon ? 1 : 0;
  p.c_vac = sqrt(h->cs2_vac);
  p.eps_cut = h->d.eps_cut;
  p.theta = h->d.theta;
  p.newton_tol = h->d.newton_tol;
  p.pi_reg = h->d.pi_reg;
  p.newton_maxit = h->d.newton_maxit;
  p.vac_zero = h->d.pi_reg > 0.0 && h->p_at0 == 0.0;
  // quiet tiles: neighbourhood radius in tiles covering 6 cells per axis
  const int td[3] = {kTiles[h->tile].tx, kTiles[h->tile].ty, kTiles[h->tile].tz};
  for (int a = 0; a < 3; ++a) p.quiet_r[a] = h->quiet_on ? (6 + td[a] - 1) / td[a] : 0;
  p.guess = h->d.guess;
  p.mlp_mfma = h->mlp_mode == KTMI_MLP_BF16;
  p.mlp = h->mlp_ok ? h->mlp_dev : nullptr;
  return p;
}

static hipEvent_t take_event(ktmi_handle* h) {
  if (!h->pool.empty()) {
    hipEvent_t e = h->pool.back();
    h->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

template <typename F>
static int launch(ktmi_handle* h, int kid, F&& body) {
  hipEvent_t a = nullptr, b = nullptr;
  if (h->timing) {
    a = take_event(h);
    b = take_event(h);
    HIP_TRY(h, hipEventRecord(a, h->stream));
  }
  body();
  HIP_TRY(h, hipGetLastError());
  if (h->timing) {
    HIP_TRY(h, hipEventRecord(b, h->stream));
    h->recs.push_back({kid, a, b});
  }
  return KTMI_OK;
}

static Geo geo(const ktmi_handle* h, double tau, double tau1) {
  Geo g;
  g.tau = tau;
  g.tau1 = tau1;
  g.cart = h->d.cartesian;
  return g;
}

// One grouped launch of a stencil pass over the events of a table that share a
// tile shape, precision and guess kind.
static const PassLauncher kPassLaunch[PASS_COUNT][2] = {
    {launch_pass0_f64, launch_pass0_f32}, {launch_pass1_f64, launch_pass1_f32},
    {launch_pass2_f64, launch_pass2_f32}, {launch_pass3_f64, launch_pass3_f32},
    {launch_pass4_f64, launch_pass4_f32}, {launch_pass5_f64, launch_pass5_f32},
    {launch_pass6_f64, launch_pass6_f32}, {launch_pass7_f64, launch_pass7_f32},
    {launch_pass8_f64, launch_pass8_f32}, {launch_pass9_f64, launch_pass9_f32},
    {launch_pass10_f64, launch_pass10_f32}};

static void launch_class(int pass, hipStream_t s, int tile, int precision, bool net,
                         const EventDesc* evs, const GroupTable& gt) {
  kPassLaunch[pass][precision == KTMI_MIXED ? 1 : 0](s, tile, net, evs, gt);
}

static GroupTable single_table(const ktmi_handle* h) {
  GroupTable gt;
  memset(&gt, 0, sizeof(gt));
  gt.nev = 1;
  gt.start[0] = 0;
  gt.start[1] = h->tg.ntiles;
  return gt;
}

static EventDesc make_event(const ktmi_handle* h) {
  EventDesc ev;
  memset(&ev, 0, sizeof(ev));
  ev.f = h->f;
  ev.p = step_params(h);
  ev.eos = h->eos;
  ev.tg = h->tg;
  ev.cart = h->d.cartesian;
  ev.viscous = h->d.viscous;
  ev.clock = h->clock;
  return ev;
}

// Uploads the handle's event table when its parameters changed.
static int upload_event(ktmi_handle* h) {
  if (!h->ev_dirty) return KTMI_OK;
  h->ev = make_event(h);
  HIP_TRY(h, hipMemcpyAsync(h->dev_ev, &h->ev, sizeof(EventDesc), hipMemcpyHostToDevice,
                            h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));  // h->ev may change before a later upload
  h->ev_dirty = false;
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  return KTMI_OK;
}

// The kernels of one step for the events of one class (same tile, precision, mode).
// mode: 0 ideal, 1 viscous (Sec. II), 2 viscous with the lambda_1 term, 3 viscous
// with bulk pressure and baryon density (no network instances: net is ignored).
static int enqueue_class_step(ktmi_handle* h, hipStream_t s, int tile, int precision, int mode,
                              bool net, const EventDesc* evs, const GroupTable& gt) {
  int rc;
  if (mode) {
    const int p1 = mode == 3 ? PASS_STAGE1_BK : (mode == 2 ? PASS_STAGE1_V_L1 : PASS_STAGE1_V);
    const int p2 = mode == 3 ? PASS_STAGE2_PI_BK : (mode == 2 ? PASS_STAGE2_PI_L1 : PASS_STAGE2_PI);
    const int p3 = mode == 3 ? PASS_STAGE2_T_BK : PASS_STAGE2_T_V;
    const bool nn = net && mode != 3;
    rc = launch(h, K_STAGE1, [&] { launch_class(p1, s, tile, precision, nn, evs, gt); });
    if (rc) return rc;
    rc = launch(h, K_STAGE2PI, [&] { launch_class(p2, s, tile, precision, false, evs, gt); });
    if (rc) return rc;
    // stage 2T starts its root solves from the predictor's e (no network)
    return launch(h, K_STAGE2T, [&] { launch_class(p3, s, tile, precision, false, evs, gt); });
  }
  rc = launch(h, K_STAGE1,
              [&] { launch_class(PASS_STAGE1_I, s, tile, precision, net, evs, gt); });
  if (rc) return rc;
  return launch(h, K_STAGE2T,
                [&] { launch_class(PASS_STAGE2_T_I, s, tile, precision, false, evs, gt); });
}

static bool uses_net(const ktmi_handle* h) { return h->d.guess == KTMI_GUESS_MLP; }

// 0 ideal, 1 viscous, 2 viscous with the lambda_1 term, 3 with bulk / baryon
static int step_mode(const ktmi_handle* h) {
  if (!h->d.viscous) return 0;
  if (has_ext(&h->d)) return 3;
  return h->d.lambda1_hat != 0.0 ? 2 : 1;
}

static int enqueue_step(ktmi_handle* h) {
  const GroupTable gt = single_table(h);
  int rc = enqueue_class_step(h, h->stream, h->tile, h->d.precision, step_mode(h), uses_net(h),
                              h->dev_ev, gt);
  if (rc) return rc;
  return launch(h, K_REDUCE, [&] {
    hipLaunchKernelGGL(k_reduce, dim3(kNP), dim3(kRedBlock), 0, h->stream, h->dev_ev);
  });
}

// Marks every tile as not quiet (the next step computes them all).
static int clear_quiet(ktmi_handle* h) {
  if (!h->bound) return KTMI_OK;
  const int n = (int)quiet_doubles(&h->d);
  hipLaunchKernelGGL(k_zero, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, h->stream,
                     (double*)h->f.quiet, n);
  HIP_TRY(h, hipGetLastError());
  return KTMI_OK;
}

static int finish_initial(ktmi_handle* h) {
  if (int rc = upload_event(h)) return rc;
  hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(64), 0, h->stream, h->clock, h->tau);
  const GroupTable gt = single_table(h);
  int rc = launch(h, K_FIRST, [&] {
    launch_class(PASS_FIRST, h->stream, h->tile, h->d.precision, false, h->dev_ev, gt);
  });
  if (rc) return rc;
  rc = launch(h, K_INIT, [&] {
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlock), 0, h->stream, h->f.acc, 32);
  });
  if (rc) return rc;
  if (int rc2 = clear_quiet(h)) return rc2;
  h->step = 0;
  h->ready = true;
  return KTMI_OK;
}

// u~ buffers of the current state (the kernels swap roles every step).
static double* const* cur_u(const ktmi_handle* h) { return (h->step & 1) ? h->f.up : h->f.u; }
static double* const* prev_u(const ktmi_handle* h) { return (h->step & 1) ? h->f.u : h->f.up; }

static int check_setup(ktmi_handle* h) {
  if (!h->bound) return fail(h, KTMI_ESTATE, "no workspace bound");
  if (!h->eos_set) return fail(h, KTMI_ESTATE, "EoS table must be set after binding");
  if (h->d.guess == KTMI_GUESS_MLP && !h->mlp_ok)
    return fail(h, KTMI_ESTATE, "guess mode KTMI_GUESS_MLP needs ktmi_set_mlp first");
  return KTMI_OK;
}


// ---------------------------------------------------------------------------
// Groups: many events stepped together.  Events are sorted into classes of
// equal (mode, precision, tile shape, guess kind); per class and stage one
// launch covers the tiles of all its events (the kernels find their event from
// the tile index), then one reduce launch serves every event.
// ---------------------------------------------------------------------------
struct ktmi_group {
  std::vector<ktmi_handle*> hs;  // in class order
  hipStream_t stream = nullptr;
  struct Class {
    int tile, precision, mode;  // mode: step_mode() of its events
    bool net;   // learned root-solve guess
    int first;  // index of the class's first event in the device table
    GroupTable gt;
  };
  std::vector<Class> classes;
  EventDesc* dev = nullptr;           // nev entries in class order
  std::vector<EventDesc> host;        // kept alive for the asynchronous upload
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  std::string err;
  ktmi_handle timing_stub;  // carries the stream and error text for launch()
};

static int group_fail(ktmi_group* g, int code, const std::string& msg) {
  g->err = msg;
  return code;
}

static int enqueue_group_step(ktmi_group* g) {
  ktmi_handle* h = &g->timing_stub;
  for (const auto& c : g->classes) {
    int rc = enqueue_class_step(h, g->stream, c.tile, c.precision, c.mode, c.net, g->dev + c.first,
                                c.gt);
    if (rc) return group_fail(g, rc, h->err);
  }
  const int nev = (int)g->hs.size();
  hipLaunchKernelGGL(k_reduce, dim3(kNP * nev), dim3(kRedBlock), 0, g->stream, g->dev);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return group_fail(g, KTMI_EHIP, hipGetErrorString(e));
  return KTMI_OK;
}

extern "C" {

void ktmi_desc_default(ktmi_desc* d) {
  memset(d, 0, sizeof(*d));
  d->eps_cut = 1e-7;
  d->theta = 1.8;
  d->newton_tol = 1e-12;
  d->newton_maxit = 100;
  d->pi_reg = 0.3;
  d->precision = KTMI_FP64;
  d->guess = KTMI_GUESS_PREV;
  d->tile = -1;
  d->taupi_coef = 5.0;
  d->lambda1_hat = 0.0;
  d->zetas = 0.0;
  d->taubulk_coef = 5.0;
  d->baryon = 0;
  d->cfl_limit = 0.5;
}

size_t ktmi_workspace_bytes(const ktmi_desc* d) {
  std::string why;
  if (!desc_ok(d, &why)) return 0;
  const size_t fs = field_stride(d);
  const size_t nb = (size_t)max_tiles(d);
  size_t bytes = (size_t)num_fields(d) * fs * sizeof(double);
  bytes += ((2 * nb * kNP + 31) / 32 * 32) * sizeof(double);  // partials
  bytes += 32 * sizeof(double);                               // accumulators
  bytes += quiet_doubles(d) * sizeof(double);                 // quiet-tile flags
  bytes += 3 * (size_t)kEosMaxRows * sizeof(double);          // EoS table
  bytes += 3 * (size_t)kEosMaxRows * sizeof(float);           // its FP32 copy
  bytes += 4096 + 512;                                         // event table, clock
  bytes += (kMlpDevBytes + 255) / 256 * 256;                   // network parameters
  bytes += (surface_scratch_words(d->nx, d->ny, d->ne) * 8 + 255) / 256 * 256;  // surface finder
  return bytes;
}

int ktmi_create(const ktmi_desc* d, ktmi_handle** out) {
  std::string why;
  if (!out) return fail(nullptr, KTMI_EINVAL, "null output pointer");
  *out = nullptr;
  if (!desc_ok(d, &why)) return fail(nullptr, KTMI_EINVAL, why);
  ktmi_handle* h = new ktmi_handle();
  h->d = *d;
  h->tau = d->tau0;
  h->nblk = num_blocks(d);
  h->tile = d->tile < 0 ? auto_tile(d) : d->tile;
  h->tg = tile_grid(d, h->tile);
  h->fstride = field_stride(d);
  h->eos.kind = 0;
  h->eos.c_sb = 47.5 * M_PI * M_PI / 30.0 / (kHbarc * kHbarc * kHbarc);
  h->eos.inv_csb = 1.0 / h->eos.c_sb;
  h->eos.inv_csb_f = (float)h->eos.inv_csb;
  h->eos_set = true;  // ideal gas until a table is set
  *out = h;
  return KTMI_OK;
}

int ktmi_bind(ktmi_handle* h, void* ws, size_t bytes, void* stream) {
  if (!h) return KTMI_EINVAL;
  const size_t need = ktmi_workspace_bytes(&h->d);
  if (!ws) return fail(h, KTMI_EINVAL, "null workspace");
  if (bytes < need) return fail(h, KTMI_EINVAL, "workspace smaller than ktmi_workspace_bytes");
  if (((uintptr_t)ws) % 256 != 0) return fail(h, KTMI_EINVAL, "workspace must be 256-byte aligned");
  if (h->ready && (char*)ws != h->ws)
    return fail(h, KTMI_ESTATE, "workspace cannot change after the initial state is set");
  if (h->eos.kind == 1 && (char*)ws != h->ws) h->eos_set = false;  // table lives in the old workspace
  if ((char*)ws != h->ws) h->mlp_ok = false;  // so do the network parameters
  h->ws = (char*)ws;
  h->ws_bytes = bytes;
  h->stream = (hipStream_t)stream;
  double* base = (double*)ws;
  const size_t fs = h->fstride;
  int q = 0;
  Fields& f = h->f;
  // pi~ and its stage-1 value are blocks of consecutive fields (the kernels
  // address a block from its first field), Pi and n right after pi~'s 10
  const int nq = has_ext(&h->d) ? 12 : 10;
  f.fstride = (long)fs;
  f.pf32 = h->d.precision == KTMI_MIXED ? 1 : 0;  // pi~ blocks in FP32 (first half of each slot)
  f.e = base + fs * q++;
  for (int m = 0; m < 3; ++m) f.u[m] = base + fs * q++;
  for (int m = 0; m < 3; ++m) f.up[m] = base + fs * q++;
  for (int m = 0; m < 12; ++m) f.pi[m] = m < nq ? base + fs * q++ : nullptr;
  for (int m = 0; m < 4; ++m) f.T[m] = base + fs * q++;
  f.e1 = base + fs * q++;
  for (int m = 0; m < 3; ++m) f.u1[m] = base + fs * q++;
  for (int m = 0; m < 12; ++m) f.pi1[m] = m < nq ? base + fs * q++ : nullptr;
  for (int m = 0; m < 4; ++m) f.T1[m] = base + fs * q++;
  double* rest = base + fs * q;
  f.partial = rest;
  rest += (2 * (size_t)max_tiles(&h->d) * kNP + 31) / 32 * 32;
  f.acc = rest;
  rest += 32;
  f.quiet = (int*)rest;  // 4 x max tiles flags
  rest += quiet_doubles(&h->d);
  h->eos_store = rest;
  rest += 3 * (size_t)kEosMaxRows;                       // FP64 table
  rest += (3 * (size_t)kEosMaxRows * sizeof(float) + 7) / 8;  // FP32 copy
  rest = (double*)(((uintptr_t)rest + 255) / 256 * 256);
  h->dev_ev = (EventDesc*)rest;
  h->clock = rest + 4096 / 8;
  h->mlp_dev = (float*)(rest + (4096 + 512) / 8);
  h->surf_blocks = (unsigned long long*)((char*)h->mlp_dev + (kMlpDevBytes + 255) / 256 * 256);
  static_assert(sizeof(EventDesc) <= 4096, "event table slot");
  h->ev_dirty = true;
  h->bound = true;
  return KTMI_OK;
}

int ktmi_set_eos_conformal(ktmi_handle* h, double c_sb) {
  if (!h) return KTMI_EINVAL;
  if (!(c_sb > 0)) return fail(h, KTMI_EINVAL, "c_sb must be > 0");
  h->eos.kind = 0;
  h->eos.c_sb = c_sb;
  h->eos.inv_csb = 1.0 / c_sb;
  h->eos.inv_csb_f = (float)(1.0 / c_sb);
  h->cs2_vac = 1.0 / 3.0;
  h->eos_p0 = 0.0;
  h->p_at0 = 0.0;
  h->eos_set = true;
  h->ev_dirty = true;
  return KTMI_OK;
}

int ktmi_set_eos_table(ktmi_handle* h, double e0, double de, int n, const double* P,
                       const double* T, const double* cs2) {
  if (!h) return KTMI_EINVAL;
  if (!h->bound) return fail(h, KTMI_ESTATE, "bind a workspace before setting a table");
  if (n < 2 || n > kEosMaxRows) return fail(h, KTMI_EINVAL, "table rows must be in [2, 8192]");
  if (!(de > 0)) return fail(h, KTMI_EINVAL, "de must be > 0");
  if (!P || !T || !cs2) return fail(h, KTMI_EINVAL, "null table column");
  const double p0 = e0 == 0.0 ? P[0] : NAN;  // P at e = 0
  if (h->quiet_on && p0 != 0.0)
    return fail(h, KTMI_ESTATE, "quiet-tile skipping needs P(0) = 0: turn it off first");
  double* dP = h->eos_store;
  double* dT = dP + kEosMaxRows;
  double* dC = dT + kEosMaxRows;
  HIP_TRY(h, hipMemcpyAsync(dP, P, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(dT, T, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(dC, cs2, sizeof(double) * n, hipMemcpyHostToDevice, h->stream));
  // FP32 copy for the mixed-precision path (rounded on the host)
  float* fP = (float*)(dC + kEosMaxRows);
  float* fT = fP + kEosMaxRows;
  float* fC = fT + kEosMaxRows;
  std::vector<float> tmp((size_t)3 * n);
  for (int i = 0; i < n; ++i) {
    tmp[i] = (float)P[i];
    tmp[(size_t)n + i] = (float)T[i];
    tmp[(size_t)2 * n + i] = (float)cs2[i];
  }
  HIP_TRY(h, hipMemcpyAsync(fP, tmp.data(), sizeof(float) * n, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(fT, tmp.data() + n, sizeof(float) * n, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(fC, tmp.data() + 2 * n, sizeof(float) * n, hipMemcpyHostToDevice,
                            h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->eos.Pf = fP;
  h->eos.Tf = fT;
  h->eos.cs2f = fC;
  h->eos.e0_f = (float)e0;
  h->eos.de_f = (float)de;
  h->eos.inv_de_f = (float)(1.0 / de);
  h->eos.kind = 1;
  h->eos.n = n;
  h->eos.e0 = e0;
  h->eos.de = de;
  h->eos.inv_de = 1.0 / de;
  h->cs2_vac = cs2[0];  // lookups clamp e = 0 to the first row
  h->eos_p0 = p0;
  h->p_at0 = P[0];
  h->eos.P = dP;
  h->eos.T = dT;
  h->eos.cs2 = dC;
  h->eos_set = true;
  h->ev_dirty = true;
  return KTMI_OK;
}

int ktmi_set_initial_primitive(ktmi_handle* h, const double* e, const double* ux,
                               const double* uy, const double* ue, const double* pi10) {
  return ktmi_set_initial_primitive_ext(h, e, ux, uy, ue, pi10, nullptr, nullptr);
}

int ktmi_set_initial_primitive_ext(ktmi_handle* h, const double* e, const double* ux,
                                   const double* uy, const double* ue, const double* pi10,
                                   const double* Pi, const double* nbar) {
  if (!h) return KTMI_EINVAL;
  if (int rc = check_setup(h)) return rc;
  if (!e || !ux || !uy || !ue) return fail(h, KTMI_EINVAL, "null field pointer");
  const size_t n = (size_t)h->d.nx * h->d.ny * h->d.ne, nb = n * sizeof(double);
  hipStream_t s = h->stream;
  HIP_TRY(h, hipMemcpyAsync(h->f.e, e, nb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(h->f.u[0], ux, nb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(h->f.u[1], uy, nb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(h->f.u[2], ue, nb, hipMemcpyDeviceToDevice, s));
  // pi~ (Pi, n) staged in FP64 in the stage-1 block; k_init_primitive stores it
  for (int m = 0; m < 10; ++m) {
    if (pi10 && h->d.viscous)
      HIP_TRY(h, hipMemcpyAsync(h->f.pi1[m], pi10 + (size_t)m * n, nb, hipMemcpyDeviceToDevice, s));
    else
      hipLaunchKernelGGL(k_zero, dim3(h->nblk), dim3(kBlock), 0, s, h->f.pi1[m], (int)n);
  }
  const bool ext = has_ext(&h->d);
  if (ext) {
    const double* src[2] = {h->d.zetas > 0.0 ? Pi : nullptr, h->d.baryon ? nbar : nullptr};
    for (int m = 0; m < 2; ++m) {
      if (src[m])
        HIP_TRY(h, hipMemcpyAsync(h->f.pi1[10 + m], src[m], n * sizeof(double), hipMemcpyDeviceToDevice, s));
      else
        hipLaunchKernelGGL(k_zero, dim3(h->nblk), dim3(kBlock), 0, s, h->f.pi1[10 + m], (int)n);
    }
  }
  h->tau = h->d.tau0;
  const StepParams p = step_params(h);
  const Geo g = geo(h, h->tau, h->tau);
  int rc = launch(h, K_INIT, [&] {
    hipLaunchKernelGGL(k_init_primitive, dim3(h->nblk), dim3(kBlock), 0, s, h->f, p, h->eos, g,
                       h->d.viscous, ext ? 1 : 0);
  });
  if (rc) return rc;
  return finish_initial(h);
}

int ktmi_set_initial_conserved(ktmi_handle* h, const double* T4, const double* pi10) {
  if (!h) return KTMI_EINVAL;
  if (int rc = check_setup(h)) return rc;
  if (!T4) return fail(h, KTMI_EINVAL, "null T pointer");
  const size_t n = (size_t)h->d.nx * h->d.ny * h->d.ne, nb = n * sizeof(double);
  hipStream_t s = h->stream;
  for (int m = 0; m < 4; ++m)
    HIP_TRY(h, hipMemcpyAsync(h->f.T[m], T4 + (size_t)m * n, nb, hipMemcpyDeviceToDevice, s));
  // pi~ staged in FP64 in the stage-1 block; k_init_conserved stores it
  for (int m = 0; m < 10; ++m) {
    if (pi10 && h->d.viscous)
      HIP_TRY(h, hipMemcpyAsync(h->f.pi1[m], pi10 + (size_t)m * n, nb, hipMemcpyDeviceToDevice, s));
    else
      hipLaunchKernelGGL(k_zero, dim3(h->nblk), dim3(kBlock), 0, s, h->f.pi1[m], (int)n);
  }
  if (has_ext(&h->d))  // Pi = n = 0
    for (int m = 10; m < 12; ++m)
      hipLaunchKernelGGL(k_zero, dim3(h->nblk), dim3(kBlock), 0, s, h->f.pi[m], (int)n);
  h->tau = h->d.tau0;
  const StepParams p = step_params(h);
  const Geo g = geo(h, h->tau, h->tau);
  int rc = launch(h, K_INIT, [&] {
    if (uses_net(h))
      hipLaunchKernelGGL(k_init_conserved<true>, dim3(h->nblk), dim3(kBlock), 0, s, h->f, p,
                         h->eos, g, h->d.viscous);
    else
      hipLaunchKernelGGL(k_init_conserved<false>, dim3(h->nblk), dim3(kBlock), 0, s, h->f, p,
                         h->eos, g, h->d.viscous);
  });
  if (rc) return rc;
  return finish_initial(h);
}

int ktmi_step(ktmi_handle* h, int nsteps) {
  if (!h) return KTMI_EINVAL;
  if (!h->ready) return fail(h, KTMI_ESTATE, "set an initial state first");
  if (nsteps < 0) return fail(h, KTMI_EINVAL, "negative step count");
  if (int rc = upload_event(h)) return rc;
  const bool graph = h->use_graph && !h->timing;
  if (graph && !h->gexec) {  // capture one step; every step issues the same launches
    hipGraph_t g = nullptr;
    HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue_step(h);
    const hipError_t ec = hipStreamEndCapture(h->stream, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return hip_fail(h, ec, "hipStreamEndCapture");
    const hipError_t ei = hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      h->gexec = nullptr;
      return hip_fail(h, ei, "hipGraphInstantiate");
    }
  }
  for (int it = 0; it < nsteps; ++it) {
    if (graph) {
      HIP_TRY(h, hipGraphLaunch(h->gexec, h->stream));
    } else if (int rc = enqueue_step(h)) {
      return rc;
    }
    h->tau += h->d.h;
    h->step++;
  }
  return KTMI_OK;
}

int ktmi_set_graph(ktmi_handle* h, int on) {
  if (!h) return KTMI_EINVAL;
  if (on && !h->stream)
    return fail(h, KTMI_EINVAL, "graph replay needs a non-default stream (bind one)");
  h->use_graph = on != 0;
  if (h->gexec) {
    (void)hipGraphExecDestroy(h->gexec);
    h->gexec = nullptr;
  }
  return KTMI_OK;
}

int ktmi_set_mlp(ktmi_handle* h, const float* params, int mode) {
  if (!h) return KTMI_EINVAL;
  if (!h->bound) return fail(h, KTMI_ESTATE, "bind a workspace before setting the network");
  if (!params) return fail(h, KTMI_EINVAL, "null parameter pointer");
  if (mode != KTMI_MLP_FP32 && mode != KTMI_MLP_BF16)
    return fail(h, KTMI_EINVAL, "mode must be KTMI_MLP_FP32 or KTMI_MLP_BF16");
  hipLaunchKernelGGL(k_mlp_pack, dim3((kMlpNParam + 255) / 256), dim3(256), 0, h->stream, params,
                     h->mlp_dev);
  HIP_TRY(h, hipGetLastError());
  h->mlp_ok = true;
  h->mlp_mode = mode;
  h->ev_dirty = true;  // the next step re-uploads the event table (and re-captures a graph)
  return KTMI_OK;
}

int ktmi_set_guess(ktmi_handle* h, int guess) {
  if (!h) return KTMI_EINVAL;
  if (guess != KTMI_GUESS_PREV && guess != KTMI_GUESS_COLD && guess != KTMI_GUESS_MLP)
    return fail(h, KTMI_EINVAL, "unknown guess mode");
  if (guess == KTMI_GUESS_MLP && !h->mlp_ok)
    return fail(h, KTMI_ESTATE, "guess mode KTMI_GUESS_MLP needs ktmi_set_mlp first");
  h->d.guess = guess;
  h->ev_dirty = true;
  return KTMI_OK;
}

int ktmi_harvest(ktmi_handle* h, double* E, double* M, double* eps) {
  if (!h) return KTMI_EINVAL;
  if (!h->ready) return fail(h, KTMI_ESTATE, "no state to harvest");
  if (!E || !M || !eps) return fail(h, KTMI_EINVAL, "null output pointer");
  const int n = h->d.nx * h->d.ny * h->d.ne;
  Fields f = h->f;
  hipLaunchKernelGGL(k_harvest, dim3(h->nblk), dim3(kBlock), 0, h->stream, f, h->clock,
                     h->d.cartesian, h->d.viscous, n, E, M, eps);
  HIP_TRY(h, hipGetLastError());
  return KTMI_OK;
}

int ktmi_read(ktmi_handle* h, int field, double* dst) {
  if (!h) return KTMI_EINVAL;
  if (!h->ready) return fail(h, KTMI_ESTATE, "no state to read");
  if (!dst) return fail(h, KTMI_EINVAL, "null destination");
  const int n = h->d.nx * h->d.ny * h->d.ne;
  const size_t nb = (size_t)n * sizeof(double);
  hipStream_t s = h->stream;
  const double* src = nullptr;
  if (field == KTMI_F_EPS)
    src = h->f.e;
  else if (field >= KTMI_F_UX && field < KTMI_F_UX + 3)
    src = cur_u(h)[field - KTMI_F_UX];
  else if (field >= KTMI_F_PI && field < KTMI_F_PI + 10) {
    hipLaunchKernelGGL(k_read_pi, dim3(h->nblk), dim3(kBlock), 0, s, h->f.e,
                       h->f.pi[field - KTMI_F_PI], dst, n, h->f.pf32);
    HIP_TRY(h, hipGetLastError());
    return KTMI_OK;
  } else if (field == KTMI_F_BULK || field == KTMI_F_NB) {
    if (has_ext(&h->d))
      hipLaunchKernelGGL(k_read_pi, dim3(h->nblk), dim3(kBlock), 0, s, h->f.e,
                         h->f.pi[10 + field - KTMI_F_BULK], dst, n, h->f.pf32);
    else
      hipLaunchKernelGGL(k_zero, dim3(h->nblk), dim3(kBlock), 0, s, dst, n);
    HIP_TRY(h, hipGetLastError());
    return KTMI_OK;
  } else if (field >= KTMI_F_T && field < KTMI_F_T + 4)
    src = h->f.T[field - KTMI_F_T];
  else if (field >= KTMI_F_UPREV && field < KTMI_F_UPREV + 3)
    src = prev_u(h)[field - KTMI_F_UPREV];
  else
    return fail(h, KTMI_EINVAL, "unknown field id");
  HIP_TRY(h, hipMemcpyAsync(dst, src, nb, hipMemcpyDeviceToDevice, s));
  return KTMI_OK;
}

int ktmi_step_until(ktmi_handle* h, double eps_stop, int max_steps, int check_every, int* taken) {
  if (!h) return KTMI_EINVAL;
  if (!taken || max_steps < 0 || check_every < 1)
    return fail(h, KTMI_EINVAL, "need taken != NULL, max_steps >= 0, check_every >= 1");
  *taken = 0;
  while (*taken < max_steps) {
    const int n = std::min(check_every, max_steps - *taken);
    if (int rc = ktmi_step(h, n)) return rc;
    *taken += n;
    ktmi_diagnostics d;
    if (int rc = ktmi_diag(h, &d)) return rc;
    if (d.eps_max < eps_stop) break;
  }
  return KTMI_OK;
}

size_t ktmi_snapshot_doubles(const ktmi_handle* h, int with_pi) {
  if (!h) return 0;
  return (size_t)(with_pi ? 14 : 4) * h->d.nx * h->d.ny * h->d.ne;
}

int ktmi_snapshot(ktmi_handle* h, double* dst, int with_pi) {
  if (!h) return KTMI_EINVAL;
  if (!dst) return fail(h, KTMI_EINVAL, "null destination");
  const size_t n = (size_t)h->d.nx * h->d.ny * h->d.ne;
  const int nf = with_pi ? 14 : 4;
  for (int f = 0; f < nf; ++f) {
    const int field = f == 0 ? KTMI_F_EPS : (f < 4 ? KTMI_F_UX + f - 1 : KTMI_F_PI + f - 4);
    if (int rc = ktmi_read(h, field, dst + f * n)) return rc;
  }
  return KTMI_OK;
}

int ktmi_surface(ktmi_handle* h, const double* A, double tau_A, const double* B, double tau_B,
                 int with_pi, double eps_f, double* out, long capacity,
                 unsigned long long* count) {
  if (!h) return KTMI_EINVAL;
  if (!A || !B || !count || capacity < 0 || (capacity > 0 && !out))
    return fail(h, KTMI_EINVAL, "null slice, count or output buffer, or capacity < 0");
  if (!(tau_B > tau_A) || !std::isfinite(eps_f))
    return fail(h, KTMI_EINVAL, "need tau_B > tau_A and a finite eps_f");
  if (!h->bound) return fail(h, KTMI_ESTATE, "bind a workspace first");
  SurfaceArgs a;
  a.nx = h->d.nx;
  a.ny = h->d.ny;
  a.ne = h->d.ne;
  a.dx = h->d.dx;
  a.dy = h->d.dy;
  a.de = h->d.de;
  a.A = A;
  a.B = B;
  a.tauA = tau_A;
  a.tauB = tau_B;
  a.nf = with_pi ? 14 : 4;
  a.eps_f = eps_f;
  a.cart = h->d.cartesian;
  a.out = out;
  a.capacity = capacity;
  a.count = count;
  a.blocks = h->surf_blocks;
  return launch(h, K_SURFACE, [&] { (void)launch_surface(a, h->stream); });
}

int ktmi_diag(ktmi_handle* h, ktmi_diagnostics* out) {
  if (!h || !out) return KTMI_EINVAL;
  if (!h->ready) return fail(h, KTMI_ESTATE, "no state");
  double acc[16];
  HIP_TRY(h, hipMemcpyAsync(acc, h->f.acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  out->tau = h->tau;
  out->step = h->step;
  out->geo_src = acc[0];
  out->max_cfl = acc[1];
  out->solves = (long)acc[2];
  out->newton_mean = acc[2] > 0 ? acc[3] / acc[2] : 0.0;
  out->newton_max = (long)acc[4];
  out->fallbacks = (long)acc[5];
  out->nonconv = (long)acc[6];
  out->nans = (long)acc[7];
  out->clamps = (long)acc[8];
  out->eps_max = acc[9];
  out->sum_Ttt = acc[10];
  out->vacuum = (long)acc[11];
  out->negative = (long)acc[12];
  out->errors = (out->nans > 0 ? KTMI_ERR_NAN : 0) | (out->negative > 0 ? KTMI_ERR_NEG_EPS : 0) |
                (out->nonconv > 0 ? KTMI_ERR_NONCONV : 0) |
                (out->max_cfl > h->d.cfl_limit ? KTMI_ERR_CFL : 0);
  return KTMI_OK;
}

int ktmi_set_timing(ktmi_handle* h, int on) {
  if (!h) return KTMI_EINVAL;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (auto& r : h->recs) {
    h->pool.push_back(r.a);
    h->pool.push_back(r.b);
  }
  h->recs.clear();
  h->timing = on != 0;
  return KTMI_OK;
}

int ktmi_kernel_count(void) { return K_COUNT; }

const char* ktmi_kernel_name(int k) { return (k >= 0 && k < K_COUNT) ? kKernelNames[k] : ""; }

int ktmi_timing(ktmi_handle* h, int k, double* total_ms, long* launches) {
  if (!h || !total_ms || !launches) return KTMI_EINVAL;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  double t = 0.0;
  long cnt = 0;
  for (auto& r : h->recs) {
    if (r.k != k) continue;
    float ms = 0.f;
    HIP_TRY(h, hipEventElapsedTime(&ms, r.a, r.b));
    t += ms;
    cnt++;
  }
  *total_ms = t;
  *launches = cnt;
  return KTMI_OK;
}

int ktmi_tile_count(void) { return kNumTiles; }

int ktmi_tile_shape(int t, int* tx, int* ty, int* tz) {
  if (t < 0 || t >= kNumTiles || !tx || !ty || !tz) return KTMI_EINVAL;
  *tx = kTiles[t].tx;
  *ty = kTiles[t].ty;
  *tz = kTiles[t].tz;
  return KTMI_OK;
}

int ktmi_get_tile(const ktmi_handle* h) { return h ? h->tile : KTMI_EINVAL; }

int ktmi_set_tile(ktmi_handle* h, int t) {
  if (!h) return KTMI_EINVAL;
  if (t < -1 || t >= kNumTiles) return fail(h, KTMI_EINVAL, "tile index out of range");
  h->tile = t < 0 ? auto_tile(&h->d) : t;
  h->tg = tile_grid(&h->d, h->tile);
  h->ev_dirty = true;
  return clear_quiet(h);  // flags are per tile of the old shape
}

int ktmi_quiet_tiles(ktmi_handle* h, long* quiet, long* total) {
  if (!h || !quiet || !total) return KTMI_EINVAL;
  if (!h->ready) return fail(h, KTMI_ESTATE, "no state");
  const int nt = h->tg.ntiles;
  std::vector<int> flags(nt);
  // the step with clock parity p writes flag buffer 1 - p: after an odd number
  // of steps the latest flags are in buffer 1
  const int* src = h->f.quiet + ((h->step & 1) ? nt : 0);
  HIP_TRY(h, hipMemcpyAsync(flags.data(), src, sizeof(int) * nt, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  long n = 0;
  for (int v : flags) n += v != 0;
  *quiet = n;
  *total = nt;
  return KTMI_OK;
}

int ktmi_set_quiet_skip(ktmi_handle* h, int on) {
  if (!h) return KTMI_EINVAL;
  if (on && h->eos_p0 != 0.0)
    return fail(h, KTMI_ESTATE, "quiet-tile skipping needs an EoS with P(0) = 0");
  h->quiet_on = on != 0;
  h->ev_dirty = true;
  return clear_quiet(h);
}

size_t ktmi_group_workspace_bytes(int nev) {
  if (nev < 1) return 0;
  return (size_t)nev * sizeof(EventDesc) + 256;
}

int ktmi_group_create(ktmi_handle* const* hs, int nev, void* ws, size_t bytes, ktmi_group** out) {
  if (!out) return fail(nullptr, KTMI_EINVAL, "null output pointer");
  *out = nullptr;
  if (!hs || nev < 1) return fail(nullptr, KTMI_EINVAL, "need at least one handle");
  if (!ws || bytes < ktmi_group_workspace_bytes(nev) || ((uintptr_t)ws) % 256)
    return fail(nullptr, KTMI_EINVAL, "group workspace too small or not 256-byte aligned");
  for (int i = 0; i < nev; ++i) {
    if (!hs[i] || !hs[i]->ready)
      return fail(nullptr, KTMI_ESTATE, "every handle needs an initial state before grouping");
    if (hs[i]->stream != hs[0]->stream)
      return fail(nullptr, KTMI_EINVAL, "all handles of a group must share one stream");
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(nullptr, KTMI_EINVAL, "a handle appears twice");
  }
  ktmi_group* g = new ktmi_group();
  g->stream = hs[0]->stream;
  g->timing_stub.stream = g->stream;
  g->dev = (EventDesc*)ws;
  // classes in first-seen order; events keep their order inside a class
  std::vector<int> order;
  std::vector<std::vector<int>> members;
  for (int i = 0; i < nev; ++i) {
    const ktmi_handle* h = hs[i];
    int c = -1;
    for (size_t k = 0; k < g->classes.size(); ++k)
      if (g->classes[k].tile == h->tile && g->classes[k].precision == h->d.precision &&
          g->classes[k].mode == step_mode(h) && g->classes[k].net == uses_net(h))
        c = (int)k;
    if (c < 0) {
      ktmi_group::Class cl{};
      cl.tile = h->tile;
      cl.precision = h->d.precision;
      cl.mode = step_mode(h);
      cl.net = uses_net(h);
      g->classes.push_back(cl);
      members.emplace_back();
      c = (int)g->classes.size() - 1;
    }
    members[c].push_back(i);
  }
  int pos = 0;
  for (size_t k = 0; k < g->classes.size(); ++k) {
    auto& cl = g->classes[k];
    if ((int)members[k].size() > kMaxGroup) {
      delete g;
      return fail(nullptr, KTMI_EINVAL, "too many events of one class (max 128)");
    }
    cl.first = pos;
    memset(&cl.gt, 0, sizeof(cl.gt));
    cl.gt.nev = (int)members[k].size();
    int t = 0;
    for (int m = 0; m < cl.gt.nev; ++m) {
      ktmi_handle* h = hs[members[k][m]];
      cl.gt.start[m] = t;
      t += h->tg.ntiles;
      g->hs.push_back(h);
      g->host.push_back(make_event(h));
      pos++;
    }
    cl.gt.start[cl.gt.nev] = t;
  }
  const hipError_t e = hipMemcpyAsync(g->dev, g->host.data(), sizeof(EventDesc) * nev,
                                      hipMemcpyHostToDevice, g->stream);
  const hipError_t e2 = e == hipSuccess ? hipStreamSynchronize(g->stream) : e;
  if (e2 != hipSuccess) {
    delete g;
    return fail(nullptr, KTMI_EHIP, std::string("group table upload: ") + hipGetErrorString(e2));
  }
  *out = g;
  return KTMI_OK;
}

int ktmi_group_step(ktmi_group* g, int nsteps) {
  if (!g) return KTMI_EINVAL;
  if (nsteps < 0) return group_fail(g, KTMI_EINVAL, "negative step count");
  if (g->use_graph && !g->gexec) {
    hipGraph_t gr = nullptr;
    hipError_t e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return group_fail(g, KTMI_EHIP, hipGetErrorString(e));
    const int rc = enqueue_group_step(g);
    e = hipStreamEndCapture(g->stream, &gr);
    if (rc) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    if (e != hipSuccess) return group_fail(g, KTMI_EHIP, hipGetErrorString(e));
    e = hipGraphInstantiate(&g->gexec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) {
      g->gexec = nullptr;
      return group_fail(g, KTMI_EHIP, hipGetErrorString(e));
    }
  }
  for (int it = 0; it < nsteps; ++it) {
    if (g->use_graph) {
      const hipError_t e = hipGraphLaunch(g->gexec, g->stream);
      if (e != hipSuccess) return group_fail(g, KTMI_EHIP, hipGetErrorString(e));
    } else if (int rc = enqueue_group_step(g)) {
      return rc;
    }
    for (ktmi_handle* h : g->hs) {
      h->tau += h->d.h;
      h->step++;
    }
  }
  return KTMI_OK;
}

int ktmi_group_set_graph(ktmi_group* g, int on) {
  if (!g) return KTMI_EINVAL;
  if (on && !g->stream) return group_fail(g, KTMI_EINVAL, "graph replay needs a non-default stream");
  g->use_graph = on != 0;
  if (g->gexec) {
    (void)hipGraphExecDestroy(g->gexec);
    g->gexec = nullptr;
  }
  return KTMI_OK;
}

int ktmi_group_class_count(const ktmi_group* g) { return g ? (int)g->classes.size() : KTMI_EINVAL; }

const char* ktmi_group_last_error(const ktmi_group* g) { return g ? g->err.c_str() : ""; }

void ktmi_group_destroy(ktmi_group* g) {
  if (!g) return;
  if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
  delete g;
}

const char* ktmi_last_error(const ktmi_handle* h) {
  return h ? h->err.c_str() : g_create_err.c_str();
}

void ktmi_destroy(ktmi_handle* h) {
  if (!h) return;
  for (auto& r : h->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : h->pool) (void)hipEventDestroy(e);
  if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
  delete h;
}

}  // extern "C"
