// ktmi.hip -- gfx950 kernels and C ABI for one RK2 step of the Kurganov-Tadmor
// scheme for (3+1)D viscous hydrodynamics in Milne coordinates
// (arXiv:1802.04449; equations of Sec. II, algorithm of Sec. III).
//
// One step is three stencil passes over the grid, FP64 structure-of-arrays
// fields with eta fastest:
//   stage1   : R_T and R_pi at tau_n from (e, u~, pi~)^n; predictor T', pi'
//              (u* = 2u^n - u^{n-1}); root solve -> (e', u~').
//   stage2pi : R_pi at tau_{n+1} from (e', u~', pi'); corrector pi^{n+1}.
//   stage2T  : R_T at tau_{n+1} from (e', u~') and pi^{n+1} (the paper's order:
//              pi first, then T); corrector T^{n+1}; root solve -> (e, u~)^{n+1}.
// Each workgroup owns a TX x TY x TZ tile of cells (one thread per cell).  For
// every axis the workgroup evaluates each face flux of its tile exactly once
// (one thread per face, results staged in LDS), then every cell takes the
// difference of its two faces.  Workgroups are mapped to tiles so that each of
// the 8 XCDs sweeps a contiguous slab of tiles (halo cells stay in that XCD's
// L2).  Each pass writes per-workgroup diagnostic partials; a one-workgroup
// reduce folds them in a fixed order, so results are bitwise reproducible.
// The caller provides all device memory; nothing here allocates.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/ktmi.h"
#include "ktmi_device.hpp"
#include "ktmi_mlp.hpp"

namespace ktmi {

constexpr int kBlock = 256;
constexpr int kNP = 12;            // diagnostic partials per workgroup

// Optional lower bound on the waves per SIMD of the stencil kernels (the
// compiler then caps their registers accordingly); 0 leaves it to the compiler.
#ifndef KTMI_WAVES_PER_EU
#define KTMI_WAVES_PER_EU 0
#endif
#if KTMI_WAVES_PER_EU > 0
#define KTMI_OCC __attribute__((amdgpu_waves_per_eu(KTMI_WAVES_PER_EU)))
#else
#define KTMI_OCC
#endif
constexpr int kEosMaxRows = 8192;  // table capacity reserved in the workspace

// Partial slots.  Sums: 0, 2, 3, 5-8, 10, 11.  Maxima: 1, 4, 9.
enum : int {
  P_GEO = 0, P_CFL = 1, P_SOLVES = 2, P_ITSUM = 3, P_ITMAX = 4, P_FALLBACK = 5,
  P_NONCONV = 6, P_NAN = 7, P_CLAMP = 8, P_EMAX = 9, P_TSUM = 10, P_VAC = 11
};
__host__ __device__ constexpr bool is_max_slot(int s) {
  return s == P_CFL || s == P_ITMAX || s == P_EMAX;
}

struct Fields {
  double* e;       // e^n, overwritten by e^{n+1} in stage2T
  double* u[3];    // u~^n
  double* up[3];   // u~^{n-1}; stage2T writes u~^{n+1} here
  double* pi[10];  // pi~^n, overwritten by pi~^{n+1} in stage2pi
  double* T[4];    // T~^{tau mu, n}, overwritten by T^{n+1} in stage2T
  double* e1;      // stage-1 prediction
  double* u1[3];
  double* pi1[10];
  double* T1[4];
  double* partial;  // [2][kNP][nblk]: stage1 then stage2T, slot-major
  double* acc;      // [16] accumulated diagnostics
};

struct Geo {
  double tau;   // stage time in the Milne factors (1 in Cartesian mode)
  double tau1;  // time of the state the stage produces
  int cart;
};

// Tile grid of one event.
struct TileGrid {
  int ntx, nty, ntz, ntiles;
};

// Everything a stencil kernel needs about one event, kept in device memory so
// that every step issues identical launches (graph replay) and one launch can
// cover the tiles of many events.  The clock (tau, step count, parity of the
// u~ / u~prev buffers) lives in the event's workspace and is advanced on the
// device by the reduce kernel at the end of every step.
struct EventDesc {
  Fields f;  // u and up as for parity 0
  StepParams p;
  EosDev eos;
  TileGrid tg;
  int cart;
  int viscous;
  double* clock;  // [0] tau, [1] steps taken, [2] parity
};

constexpr int kMaxGroup = 128;  // events per grouped launch
struct GroupTable {
  int nev;
  int start[kMaxGroup + 1];  // first tile of each event in the launch
};

// Per-block view of its event.  stage2 = 0: tau = tau_n, tau1 = tau_n + h;
// stage2 = 1: tau = tau1 = tau_n + h.
struct Ctx {
  Fields f;
  StepParams p;
  EosDev eos;
  TileGrid tg;
  Geo g;
  int tile;  // tile index inside the event
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Workgroups are dispatched to the 8 XCDs round robin (block b -> XCD b % 8).
// Give XCD x a contiguous range of tile ids so neighbouring tiles share its L2.
__device__ __forceinline__ int tile_of_block(int nb) {
  const int b = blockIdx.x, x = b & 7, k = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return x * per + (x < rem ? x : rem) + k;
}

// Starting point of the root solve of K = (E, K1, K2, K3): the previous
// stage's e, E itself (cold), or (NET kernels only) the network's guess.
// Every lane of the wave calls it (the matrix-core forward runs on whole
// waves); lanes with act = false only take part.  The guess mode is uniform
// over a workgroup.  The network lives in separate kernel instances (NET) so
// that its registers do not lower the occupancy of the others.
template <bool NET>
__device__ __forceinline__ double root_guess(const StepParams& p, bool act, double E, double K1,
                                             double K2, double K3, double prev) {
  if (NET && p.guess == KTMI_GUESS_MLP) {
    const double M2 = K1 * K1 + K2 * K2 + K3 * K3;
    const bool use = act && E >= p.eps_cut && E < 1e300 && M2 < 1e300;
    if (p.mlp_mfma) {
      if (__ballot(use) == 0) return prev;
      const double g = mlp_guess_wave(p.mlp, reinterpret_cast<const uint16_t*>(p.mlp + kMlpPad),
                                      use ? E : 1.0, use ? M2 : 0.0);
      return use ? g : prev;
    }
    return use ? mlp_guess_lane(p.mlp, E, M2) : prev;
  }
  return p.guess == KTMI_GUESS_COLD ? E : prev;
}

// Position of this thread's cell.
struct Pos {
  int i, j, k;     // global cell coordinates
  int lx, ly, lz;  // coordinates inside the tile
  int i0, j0, k0;  // tile origin
  int c;           // flat index (valid only if active)
  bool active;
};

__device__ __forceinline__ Ctx load_ctx(const EventDesc* __restrict__ evs, const GroupTable& gt,
                                        int stage2) {
  const int t = tile_of_block(gt.start[gt.nev]);
  int e = 0;
  while (e + 1 < gt.nev && t >= gt.start[e + 1]) ++e;
  const EventDesc& E = evs[e];
  Ctx c;
  c.f = E.f;
  c.p = E.p;
  c.eos = E.eos;
  c.tg = E.tg;
  const double tau = E.clock[0];
  const bool odd = E.clock[2] != 0.0;
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    c.f.u[m] = odd ? E.f.up[m] : E.f.u[m];
    c.f.up[m] = odd ? E.f.u[m] : E.f.up[m];
  }
  c.g.cart = E.cart;
  c.g.tau1 = tau + E.p.h;
  c.g.tau = stage2 ? c.g.tau1 : tau;
  c.tile = t - gt.start[e];
  return c;
}

template <int TX, int TY, int TZ>
__device__ __forceinline__ Pos cell_pos(const StepParams& p, const TileGrid& tg, int t) {
  Pos q;
  const int tk = t % tg.ntz, r = t / tg.ntz;
  const int tj = r % tg.nty, ti = r / tg.nty;
  q.i0 = ti * TX;
  q.j0 = tj * TY;
  q.k0 = tk * TZ;
  const int tid = threadIdx.x;
  q.lz = tid % TZ;
  q.ly = (tid / TZ) % TY;
  q.lx = tid / (TZ * TY);
  q.i = q.i0 + q.lx;
  q.j = q.j0 + q.ly;
  q.k = q.k0 + q.lz;
  q.active = tid < TX * TY * TZ && q.i < p.nx && q.j < p.ny && q.k < p.ne;
  q.c = (q.i * p.ny + q.j) * p.ne + q.k;
  return q;
}

// pi~ at a cell: PI_SRC 0 -> 0, 1 -> zero where e == 0 (vacuum), 2 -> as stored.
template <int PI_SRC>
__device__ __forceinline__ double ld_pi(const double* const* pi, int m, int idx, double e) {
  if (PI_SRC == 0) return 0.0;
  const double v = pi[m][idx];
  if (PI_SRC == 1) return e == 0.0 ? 0.0 : v;
  return v;
}

// KT face flux H = [F(Q^r) + F(Q^l)]/2 - c (Q^r - Q^l)/2 (Sec. III, eq. flux_out)
// at the face between cells a and a+1 along `axis` (1 = x, 2 = y, 3 = eta).
// `base` is the flat index of the row's cell with coordinate 0 along the axis.
// Components 0..3: T~^{d nu} part (if DO_T); 4..13: u~^d pi~ part (if DO_PI).
// Returns the face's local speed c.  A face whose four stencil cells are exact
// vacuum (all primitives zero) has H = 0 and c = c_vac, so it skips the arithmetic.
// R is the arithmetic type (double, or float on the mixed-precision path).
template <typename R, bool DO_T, bool DO_PI, int PI_SRC>
__device__ __forceinline__ R face_flux(const double* __restrict__ e, const double* const* u,
                                       const double* const* pi, int base, int a, int n,
                                       int stride, int axis, R tauf, const StepParams& p,
                                       const EosDev& eos, R H[14]) {
  int idx[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) idx[t] = base + clampi(a - 1 + t, 0, n - 1) * stride;
  // Vacuum faces skip all arithmetic.  Every state the kernels write has u~ = 0
  // where e = 0 (the root solve and the cutoff return all-zero primitives), and
  // with PI_SRC 0/1 pi~ reads as zero there too, so e alone decides: it is
  // loaded first and a vacuum face skips the other loads.  As-stored pi~
  // (PI_SRC 2) can be nonzero where e = 0, so there the whole stencil is loaded
  // at once (no dependent second round of loads) and e and pi~ decide.
  double ev[4];
  bool vac = true;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    ev[t] = e[idx[t]];
    vac = vac && (ev[t] == 0.0);
  }
  R q4[14][4];
  if (PI_SRC == 2) {
#pragma unroll
    for (int m = 0; m < 10; ++m)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double x = pi[m][idx[t]];
        vac = vac && (x == 0.0);
        q4[4 + m][t] = (R)x;
      }
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int t = 0; t < 4; ++t) q4[1 + m][t] = (R)u[m][idx[t]];
  }
  if (vac) {
#pragma unroll
    for (int k = 0; k < 14; ++k) H[k] = R(0);
    return (R)p.c_vac;
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) q4[0][t] = (R)ev[t];
  if (PI_SRC != 2) {
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int t = 0; t < 4; ++t) q4[1 + m][t] = (R)u[m][idx[t]];
#pragma unroll
    for (int m = 0; m < 10; ++m)
#pragma unroll
      for (int t = 0; t < 4; ++t) q4[4 + m][t] = (R)ld_pi<PI_SRC>(pi, m, idx[t], ev[t]);
  }
  R qL[14], qR[14];
  const R th = (R)p.theta;
#pragma unroll
  for (int v = 0; v < 14; ++v) {
    const R a0 = q4[v][0], a1 = q4[v][1], a2 = q4[v][2], a3 = q4[v][3];
    qL[v] = a1 + R(0.5) * mm_slope_r<R>(th, a0, a1, a2);
    qR[v] = a2 - R(0.5) * mm_slope_r<R>(th, a1, a2, a3);
  }
  R QL[14], FL[14], QR[14], FR[14], sL, sR;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const R* q = side ? qR : qL;
    R* Q = side ? QR : QL;
    R* F = side ? FR : FL;
    const R ux = q[1], uy = q[2], ue = q[3];
    const R ut = sqrt(R(1) + ux * ux + uy * uy + ue * ue);
    R P, cs2;
    eos_p_cs2_r<R>(eos, q[0], P, cs2);
    const R w = (q[0] > R(0) ? q[0] : R(0)) + P;
    const R u4[4] = {ut, ux, uy, ue};
    const R ud = u4[axis];
    if (DO_T) {
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) {
        Q[nu] = tauf * (w * ut * u4[nu] - (nu == 0 ? P : R(0)) + q[4 + sym(0, nu)]);
        F[nu] = tauf * (w * ud * u4[nu] + (nu == axis ? P : R(0)) + q[4 + sym(axis, nu)]);
      }
    }
    if (DO_PI) {
#pragma unroll
      for (int m = 0; m < 10; ++m) {
        Q[4 + m] = ut * q[4 + m];
        F[4 + m] = ud * q[4 + m];
      }
    }
    const R s = local_speed_r<R>(ut, ux, uy, ue, ud, cs2);
    if (side)
      sR = s;
    else
      sL = s;
  }
  const R c = fmax(sL, sR);
#pragma unroll
  for (int k = 0; k < 14; ++k) {
    const bool on = k < 4 ? DO_T : DO_PI;
    H[k] = on ? R(0.5) * (FL[k] + FR[k]) - R(0.5) * c * (QR[k] - QL[k]) : R(0);
  }
  return c;
}

// KT flux divergence of the thread's cell over all three axes (Sec. III, eq. kt):
// R[q] = -sum_d (H_{+1/2} - H_{-1/2}) / Delta_d.  Every face of the tile is
// computed once by one thread and staged in LDS (component-major).  Returns
// max over the computed faces of c / Delta (for the CFL diagnostic).
template <typename RT, int TX, int TY, int TZ, bool DO_T, bool DO_PI, int PI_SRC>
__device__ __forceinline__ double tile_divergence(const double* __restrict__ e,
                                                  const double* const* u, const double* const* pi,
                                                  const StepParams& p, const EosDev& eos,
                                                  double tauf, const Pos& q, double R[14],
                                                  RT* lds) {
  constexpr int N = TX * TY * TZ;
#pragma unroll
  for (int k = 0; k < 14; ++k) R[k] = 0.0;
  double cfl = 0.0;
  const int tid = threadIdx.x;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int nd = d == 0 ? p.nx : (d == 1 ? p.ny : p.ne);
    if (nd == 1) continue;  // both faces see identical states: zero divergence
    constexpr int dummy = 0;
    (void)dummy;
    const int Td = d == 0 ? TX : (d == 1 ? TY : TZ);
    const int F = (Td + 1) * (N / Td);
    const double inv_del = d == 0 ? p.inv_dx : (d == 1 ? p.inv_dy : p.inv_de / tauf);
    const int stride = d == 0 ? p.ny * p.ne : (d == 1 ? p.ne : 1);
    for (int f = tid; f < F; f += kBlock) {
      // face f -> (a: position along the axis in [0, Td], lx/ly/lz of the other axes);
      // the ordering keeps eta fastest among consecutive threads where possible
      int a, fx, fy, fz;
      if (d == 0) {
        a = f / (TY * TZ);
        const int o = f % (TY * TZ);
        fx = 0; fy = o / TZ; fz = o % TZ;
      } else if (d == 1) {
        fx = f / ((TY + 1) * TZ);
        const int o = f % ((TY + 1) * TZ);
        a = o / TZ; fy = 0; fz = o % TZ;
      } else {
        const int o = f / (TZ + 1);
        a = f % (TZ + 1);
        fx = o / TY; fy = o % TY; fz = 0;
      }
      const int gi = q.i0 + fx, gj = q.j0 + fy, gk = q.k0 + fz;
      const int ga = (d == 0 ? q.i0 : (d == 1 ? q.j0 : q.k0)) + a;  // right cell of the face
      const bool inrow = (d == 0 || gi < p.nx) && (d == 1 || gj < p.ny) && (d == 2 || gk < p.ne);
      RT H[14];
      if (inrow && ga <= nd) {
        const int base = d == 0 ? (gj * p.ne + gk)
                                : (d == 1 ? (gi * p.ny) * p.ne + gk : (gi * p.ny + gj) * p.ne);
        const RT c = face_flux<RT, DO_T, DO_PI, PI_SRC>(e, u, pi, base, ga - 1, nd, stride, d + 1,
                                                        (RT)tauf, p, eos, H);
        cfl = fmax(cfl, (double)c * inv_del);
      } else {
#pragma unroll
        for (int k = 0; k < 14; ++k) H[k] = RT(0);
      }
#pragma unroll
      for (int k = 0; k < 14; ++k) lds[k * F + f] = H[k];
    }
    __syncthreads();
    if (q.active) {
      int fm, fp;
      if (d == 0) {
        fm = q.lx * (TY * TZ) + q.ly * TZ + q.lz;
        fp = fm + TY * TZ;
      } else if (d == 1) {
        fm = q.lx * ((TY + 1) * TZ) + q.ly * TZ + q.lz;
        fp = fm + TZ;
      } else {
        fm = (q.lx * TY + q.ly) * (TZ + 1) + q.lz;
        fp = fm + 1;
      }
      const RT rinv = (RT)inv_del;
#pragma unroll
      for (int k = 0; k < 14; ++k) R[k] -= (double)((lds[k * F + fp] - lds[k * F + fm]) * rinv);
    }
    __syncthreads();
  }
  (void)N;
  return cfl;
}

template <int TX, int TY, int TZ>
constexpr int lds_doubles() {
  constexpr int N = TX * TY * TZ;
  constexpr int fx = (TX + 1) * (N / TX), fy = (TY + 1) * (N / TY), fz = (TZ + 1) * (N / TZ);
  constexpr int m = fx > fy ? (fx > fz ? fx : fz) : (fy > fz ? fy : fz);
  return 14 * m;
}

// u~^tau of spatial components.
__device__ __forceinline__ double utau(double a, double b, double c) {
  return sqrt(1.0 + a * a + b * b + c * c);
}

// Israel-Stewart source (Sec. II, eqns. pitilde, Ipi; eqn. pimn with lambda_i = 0,
// tau_pi = 5 eta_v/(T s)):
// S = -(pi - eta sigma)/tau_pi - pi theta/3 - (u b + b u) - pi u~^tau/tau - I,
// sigma~, theta, D~u~ from nabla~_mu u~^nu (eq. dtuz), b^nu = pi^{nu beta} g_{beta beta} a^beta.
// uE/uL: time levels for d_tau u~.  With eta = (eta/s)(e+P) hbarc/T and
// tau_pi = 5 (eta/s) hbarc/T, eta/tau_pi = (e+P)/5.
template <typename R>
__device__ __forceinline__ void pi_source(const double* const* u, const double* const* uE,
                                          const double* const* uL, const StepParams& p,
                                          const EosDev& eos, const Geo& g, const Pos& q,
                                          double ec_d, const double pc_d[10], double S_d[10]) {
  const R ec = (R)ec_d;
  R pc[10];
#pragma unroll
  for (int m = 0; m < 10; ++m) pc[m] = (R)pc_d[m];
  const int c0 = q.c;
  const int cart = g.cart;
  const R inv_tau = (R)(1.0 / g.tau);
  const R u1c = (R)u[0][c0], u2c = (R)u[1][c0], u3c = (R)u[2][c0];
  const R uc[4] = {sqrt(R(1) + u1c * u1c + u2c * u2c + u3c * u3c), u1c, u2c, u3c};
  R G[4][4];
  {
    const R a1 = (R)uE[0][c0], a2 = (R)uE[1][c0], a3 = (R)uE[2][c0];
    const R b1 = (R)uL[0][c0], b2 = (R)uL[1][c0], b3 = (R)uL[2][c0];
    const R ea[4] = {sqrt(R(1) + a1 * a1 + a2 * a2 + a3 * a3), a1, a2, a3};
    const R eb[4] = {sqrt(R(1) + b1 * b1 + b2 * b2 + b3 * b3), b1, b2, b3};
    const R ih = (R)p.inv_h;
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) G[0][nu] = (eb[nu] - ea[nu]) * ih;
  }
  const int n3[3] = {p.nx, p.ny, p.ne};
  const int co[3] = {q.i, q.j, q.k};
  const int st[3] = {p.ny * p.ne, p.ne, 1};
  const R ihalf[3] = {(R)(0.5 * p.inv_dx), (R)(0.5 * p.inv_dy),
                      (R)(0.5 * p.inv_de * (cart ? 1.0 : 1.0 / g.tau))};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ip = c0 + (clampi(co[d] + 1, 0, n3[d] - 1) - co[d]) * st[d];
    const int im = c0 + (clampi(co[d] - 1, 0, n3[d] - 1) - co[d]) * st[d];
    const R p1 = (R)u[0][ip], p2 = (R)u[1][ip], p3 = (R)u[2][ip];
    const R m1 = (R)u[0][im], m2 = (R)u[1][im], m3 = (R)u[2][im];
    const R up4[4] = {sqrt(R(1) + p1 * p1 + p2 * p2 + p3 * p3), p1, p2, p3};
    const R um4[4] = {sqrt(R(1) + m1 * m1 + m2 * m2 + m3 * m3), m1, m2, m3};
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) G[d + 1][nu] = (up4[nu] - um4[nu]) * ihalf[d];
  }
  if (!cart) {
    G[3][0] += uc[3] * inv_tau;
    G[3][3] += uc[0] * inv_tau;
  }
  const R theta = G[0][0] + G[1][1] + G[2][2] + G[3][3];
  R a[4];
#pragma unroll
  for (int nu = 0; nu < 4; ++nu)
    a[nu] = uc[0] * G[0][nu] + uc[1] * G[1][nu] + uc[2] * G[2][nu] + uc[3] * G[3][nu];
  const R gt[4] = {R(1), R(-1), R(-1), R(-1)};
  R b[4];
#pragma unroll
  for (int nu = 0; nu < 4; ++nu)
    b[nu] = pc[sym(nu, 0)] * a[0] - pc[sym(nu, 1)] * a[1] - pc[sym(nu, 2)] * a[2] -
            pc[sym(nu, 3)] * a[3];
  R P, T;
  eos_p_t_r<R>(eos, ec, P, T);
  const R inv_taupi = T * (R)p.inv_taupi_coef;
  const R eta_over_taupi = R(0.2) * (ec + P);
  const R ue = uc[3];
  const R third = R(1) / R(3);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
    for (int nu = mu; nu < 4; ++nu) {
      const int m = sym(mu, nu);
      const R gmn = (mu == nu) ? gt[mu] : R(0);
      const R sig = gt[mu] * G[mu][nu] + gt[nu] * G[nu][mu] - uc[mu] * a[nu] -
                    uc[nu] * a[mu] - R(2) * third * (gmn - uc[mu] * uc[nu]) * theta;
      R s = -pc[m] * inv_taupi + eta_over_taupi * sig - pc[m] * theta * third -
            (uc[mu] * b[nu] + uc[nu] * b[mu]);
      if (!cart) {
        R I = R(0);  // Christoffel terms I^{mu nu}
        if (m == 0 || m == 9) I = R(2) * ue * pc[3];
        else if (m == 1) I = ue * pc[6];
        else if (m == 2) I = ue * pc[8];
        else if (m == 3) I = ue * (pc[0] + pc[9]);
        else if (m == 6) I = ue * pc[1];
        else if (m == 8) I = ue * pc[2];
        s += -(pc[m] * uc[0] + I) * inv_tau;
      }
      S_d[m] = (double)s;
    }
  }
}

// Scale pi~ so that sqrt(|pi~:pi~|) <= pi_reg (e+P); zero it where e+P = 0.
__device__ __forceinline__ void regulate(const EosDev& eos, const StepParams& p, double e,
                                         double pv[10]) {
  if (!(p.pi_reg > 0.0)) return;
  double P, c;
  eos_p_cs2(eos, e, P, c);
  const double w = (e > 0.0 ? e : 0.0) + P;
  if (!(w > 0.0)) {
#pragma unroll
    for (int m = 0; m < 10; ++m) pv[m] = 0.0;
    return;
  }
  // g~ g~ pi pi: diagonal tt/xx/yy/ee once, off-diagonals twice with sign g_mu g_nu
  const double pp = pv[0] * pv[0] + pv[4] * pv[4] + pv[7] * pv[7] + pv[9] * pv[9] -
                    2.0 * (pv[1] * pv[1] + pv[2] * pv[2] + pv[3] * pv[3]) +
                    2.0 * (pv[5] * pv[5] + pv[6] * pv[6] + pv[8] * pv[8]);
  const double rho = sqrt(fabs(pp)) / w;
  if (rho > p.pi_reg) {
    const double f = p.pi_reg / rho;
#pragma unroll
    for (int m = 0; m < 10; ++m) pv[m] *= f;
  }
}

// ---------------------------------------------------------------------------
// Workgroup reduction of the diagnostic partials (wave64 shuffles, then LDS).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void block_partials(double v[kNP], double* out, int ntiles, int tile) {
  __shared__ double red[kBlock / 64][kNP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < kNP; ++s) {
    double x = v[s];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double y = __shfl_xor(x, off, 64);
      x = is_max_slot(s) ? fmax(x, y) : x + y;
    }
    if (lane == 0) red[wave][s] = x;
  }
  __syncthreads();
  if (threadIdx.x < kNP) {
    const int s = threadIdx.x;
    double x = red[0][s];
    for (int w = 1; w < kBlock / 64; ++w) x = is_max_slot(s) ? fmax(x, red[w][s]) : x + red[w][s];
    out[(size_t)s * ntiles + tile] = x;  // slot-major: the reduce reads coalesced
  }
}

__device__ __forceinline__ void count_solve(double v[kNP], int it, int fl) {
  if (fl & kNan) v[P_NAN] += 1.0;
  if (it == 0) return;  // decided before iterating (vacuum or NaN input)
  v[P_SOLVES] += 1.0;
  v[P_ITSUM] += (double)it;
  v[P_ITMAX] = fmax(v[P_ITMAX], (double)it);
  if (fl & kFallback) v[P_FALLBACK] += 1.0;
  if (fl & kNonconv) v[P_NONCONV] += 1.0;
  if (fl & kClamp) v[P_CLAMP] += 1.0;
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Initial primitive state: cutoff, then T~^{tau mu} = tau0 Tc^{tau mu}(e, u~, pi~).
__global__ __launch_bounds__(kBlock) void k_init_primitive(Fields f, StepParams p, EosDev eos,
                                                            Geo g, int visc) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= p.ncell) return;
  double e = f.e[c];
  double u1 = f.u[0][c], u2 = f.u[1][c], u3 = f.u[2][c];
  double pv[10];
#pragma unroll
  for (int m = 0; m < 10; ++m) pv[m] = visc ? f.pi[m][c] : 0.0;
  if (!(e >= p.eps_cut)) {
    e = 0.0;
    u1 = u2 = u3 = 0.0;
#pragma unroll
    for (int m = 0; m < 10; ++m) pv[m] = 0.0;
  }
  double P, cs2;
  eos_p_cs2(eos, e, P, cs2);
  const double ut = utau(u1, u2, u3);
  const double w = e + P;
  const double tf = g.cart ? 1.0 : g.tau;
  const double u4[4] = {ut, u1, u2, u3};
  f.e[c] = e;
  f.u[0][c] = u1;
  f.u[1][c] = u2;
  f.u[2][c] = u3;
#pragma unroll
  for (int m = 0; m < 10; ++m) f.pi[m][c] = pv[m];
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) f.T[nu][c] = tf * (w * ut * u4[nu] - (nu == 0 ? P : 0.0) + pv[nu]);
}

// Initial conserved state: root solve of K = T~/tau0 - pi~^{tau .} from E.
template <bool NET>
__global__ __launch_bounds__(kBlock) void k_init_conserved(Fields f, StepParams p, EosDev eos,
                                                            Geo g, int visc) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  const bool act = c < p.ncell;  // no early exit: root_guess needs whole waves
  const double tf = g.cart ? 1.0 : g.tau;
  double pv[10], K0 = 1.0, K1 = 0.0, K2 = 0.0, K3 = 0.0;
  if (act) {
#pragma unroll
    for (int m = 0; m < 10; ++m) pv[m] = visc ? f.pi[m][c] : 0.0;
    K0 = f.T[0][c] / tf - pv[0];
    K1 = f.T[1][c] / tf - pv[1];
    K2 = f.T[2][c] / tf - pv[2];
    K3 = f.T[3][c] / tf - pv[3];
  }
  // no previous stage here: the cold start E unless the network guesses
  const double x0 = root_guess<NET>(p, act, K0, K1, K2, K3, K0);
  if (!act) return;
  int it, fl;
  const Prim s = con2prim(eos, p, K0, K1, K2, K3, x0, it, fl);
  f.e[c] = s.e;
  f.u[0][c] = s.u1;
  f.u[1][c] = s.u2;
  f.u[2][c] = s.u3;
  if (s.e == 0.0 || !visc)
#pragma unroll
    for (int m = 0; m < 10; ++m) f.pi[m][c] = 0.0;
}

// First step: u*1 from one ideal forward-Euler step; u~^{-1} = 2 u~^0 - u*1.
template <typename RT, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_first_estimate(const EventDesc* __restrict__ evs,
                                                            GroupTable gt) {
  __shared__ RT lds[lds_doubles<TX, TY, TZ>()];
  const Ctx cx = load_ctx(evs, gt, 0);
  const Fields& f = cx.f;
  const StepParams& p = cx.p;
  const EosDev& eos = cx.eos;
  const Geo& g = cx.g;
  const Pos q = cell_pos<TX, TY, TZ>(p, cx.tg, cx.tile);
  const double tf = g.cart ? 1.0 : g.tau;
  double R[14];
  tile_divergence<RT, TX, TY, TZ, true, false, 0>(f.e, f.u, f.pi, p, eos, tf, q, R, lds);
  const int c = q.c;
  double K[4] = {1.0, 0.0, 0.0, 0.0}, e = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
  if (q.active) {
    e = f.e[c];
    u1 = f.u[0][c];
    u2 = f.u[1][c];
    u3 = f.u[2][c];
    const double ut = utau(u1, u2, u3);
    double P, cs2;
    eos_p_cs2(eos, e, P, cs2);
    const double w = (e > 0.0 ? e : 0.0) + P;
    if (!g.cart) {
      R[0] += -(w * u3 * u3 + P);
      R[3] += -(w * ut * u3);
    }
    const double u4[4] = {ut, u1, u2, u3};
    const double inv_tf1 = 1.0 / (g.cart ? 1.0 : g.tau1);
#pragma unroll
    for (int nu = 0; nu < 4; ++nu)
      K[nu] = (tf * (w * ut * u4[nu] - (nu == 0 ? P : 0.0)) + p.h * R[nu]) * inv_tf1;
  }
  // the current e is a close start; the network is not used here
  const double x0 = root_guess<false>(p, q.active, K[0], K[1], K[2], K[3], e);
  if (!q.active) return;
  int it, fl;
  const Prim s = con2prim(eos, p, K[0], K[1], K[2], K[3], x0, it, fl);
  f.up[0][c] = 2.0 * u1 - s.u1;
  f.up[1][c] = 2.0 * u2 - s.u2;
  f.up[2][c] = 2.0 * u3 - s.u3;
}

// Stage 1 at tau_n (predictor) for the ideal (VISC = false) or viscous path.
template <typename RT, int TX, int TY, int TZ, bool VISC, bool NET>
__global__ __launch_bounds__(kBlock) KTMI_OCC void k_stage1(const EventDesc* __restrict__ evs,
                                                    GroupTable gt) {
  __shared__ RT lds[lds_doubles<TX, TY, TZ>()];
  const Ctx cx = load_ctx(evs, gt, 0);
  const Fields& f = cx.f;
  const StepParams& p = cx.p;
  const EosDev& eos = cx.eos;
  const Geo& g = cx.g;
  const Pos q = cell_pos<TX, TY, TZ>(p, cx.tg, cx.tile);
  double v[kNP];
#pragma unroll
  for (int s = 0; s < kNP; ++s) v[s] = 0.0;
  const double tf = g.cart ? 1.0 : g.tau;
  double R[14];
  const double cfl =
      tile_divergence<RT, TX, TY, TZ, true, VISC, VISC ? 1 : 0>(f.e, f.u, f.pi, p, eos, tf, q, R, lds);
  v[P_CFL] = cfl * p.h;
  double K[4] = {1.0, 0.0, 0.0, 0.0}, prev = 0.0;
  if (q.active) {
    const int c = q.c;
    const double e = f.e[c], u1 = f.u[0][c], u2 = f.u[1][c], u3 = f.u[2][c];
    const double ut = utau(u1, u2, u3);
    double pc[10];
#pragma unroll
    for (int m = 0; m < 10; ++m) pc[m] = VISC ? (e == 0.0 ? 0.0 : f.pi[m][c]) : 0.0;
    if (!g.cart) {  // geometric source S_T = (-Tc^{ee}, 0, 0, -Tc^{te})
      double P, cs2;
      eos_p_cs2(eos, e, P, cs2);
      const double w = (e > 0.0 ? e : 0.0) + P;
      const double see = -(w * u3 * u3 + P + pc[9]);
      R[0] += see;
      R[3] += -(w * ut * u3 + pc[3]);
      v[P_GEO] = see;
    }
    double p1[10];
    if (VISC) {
      if (e >= p.eps_cut) {
        double S[10];
        pi_source<RT>(f.u, f.up, f.u, p, eos, g, q, e, pc, S);
#pragma unroll
        for (int m = 0; m < 10; ++m) R[4 + m] += S[m];
      }
      const double s1 = 2.0 * u1 - f.up[0][c], s2 = 2.0 * u2 - f.up[1][c],
                   s3 = 2.0 * u3 - f.up[2][c];
      const double inv_uts = 1.0 / utau(s1, s2, s3);
#pragma unroll
      for (int m = 0; m < 10; ++m) p1[m] = (ut * pc[m] + p.h * R[4 + m]) * inv_uts;
      regulate(eos, p, e, p1);
#pragma unroll
      for (int m = 0; m < 10; ++m) f.pi1[m][c] = p1[m];
    } else {
#pragma unroll
      for (int m = 0; m < 10; ++m) p1[m] = 0.0;
    }
    double T1[4];
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
      T1[nu] = f.T[nu][c] + p.h * R[nu];
      f.T1[nu][c] = T1[nu];
    }
    const double inv_tf1 = 1.0 / (g.cart ? 1.0 : g.tau1);
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) K[nu] = T1[nu] * inv_tf1 - p1[nu];
    prev = e;
  }
  const double x0 = root_guess<NET>(p, q.active, K[0], K[1], K[2], K[3], prev);
  if (q.active) {
    const int c = q.c;
    int it, fl;
    const Prim s = con2prim(eos, p, K[0], K[1], K[2], K[3], x0, it, fl);
    count_solve(v, it, fl);
    f.e1[c] = s.e;
    f.u1[0][c] = s.u1;
    f.u1[1][c] = s.u2;
    f.u1[2][c] = s.u3;
  }
  block_partials(v, f.partial, cx.tg.ntiles, cx.tile);
}

// Stage 2, part 1 (tau_{n+1}): pi^{n+1} = [ (u^n pi^n + u* pi')/2 + h/2 R_pi(e', u', pi') ] / u'^tau.
template <typename RT, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) KTMI_OCC void k_stage2_pi(const EventDesc* __restrict__ evs,
                                                      GroupTable gt) {
  __shared__ RT lds[lds_doubles<TX, TY, TZ>()];
  const Ctx cx = load_ctx(evs, gt, 1);
  const Fields& f = cx.f;
  const StepParams& p = cx.p;
  const EosDev& eos = cx.eos;
  const Geo& g = cx.g;
  const Pos q = cell_pos<TX, TY, TZ>(p, cx.tg, cx.tile);
  const double tf = g.cart ? 1.0 : g.tau;
  double R[14];
  tile_divergence<RT, TX, TY, TZ, false, true, 2>(f.e1, f.u1, f.pi1, p, eos, tf, q, R, lds);
  if (!q.active) return;
  const int c = q.c;
  const double e1 = f.e1[c];
  double pc[10];
#pragma unroll
  for (int m = 0; m < 10; ++m) pc[m] = f.pi1[m][c];
  if (e1 >= p.eps_cut) {
    double S[10];
    pi_source<RT>(f.u1, f.u, f.u1, p, eos, g, q, e1, pc, S);
#pragma unroll
    for (int m = 0; m < 10; ++m) R[4 + m] += S[m];
  }
  const double en = f.e[c];
  const double a1 = f.u[0][c], a2 = f.u[1][c], a3 = f.u[2][c];
  const double utn = utau(a1, a2, a3);
  const double uts = utau(2.0 * a1 - f.up[0][c], 2.0 * a2 - f.up[1][c], 2.0 * a3 - f.up[2][c]);
  const double inv_ut1 = 1.0 / utau(f.u1[0][c], f.u1[1][c], f.u1[2][c]);
  double pn[10];
#pragma unroll
  for (int m = 0; m < 10; ++m) {
    const double pin = en == 0.0 ? 0.0 : f.pi[m][c];
    pn[m] = (0.5 * (utn * pin + uts * pc[m]) + 0.5 * p.h * R[4 + m]) * inv_ut1;
  }
  regulate(eos, p, e1, pn);
#pragma unroll
  for (int m = 0; m < 10; ++m) f.pi[m][c] = pn[m];
}

// Stage 2, part 2 (tau_{n+1}): T^{n+1} = T^n + [(T' - T^n) + h R_T(e', u', pi^{n+1})]/2,
// root solve -> (e, u~)^{n+1} (written over e^n and u~^{n-1}), diagnostics.
template <typename RT, int TX, int TY, int TZ, bool VISC, bool NET>
__global__ __launch_bounds__(kBlock) KTMI_OCC void k_stage2_T(const EventDesc* __restrict__ evs,
                                                     GroupTable gt) {
  __shared__ RT lds[lds_doubles<TX, TY, TZ>()];
  const Ctx cx = load_ctx(evs, gt, 1);
  const Fields& f = cx.f;
  const StepParams& p = cx.p;
  const EosDev& eos = cx.eos;
  const Geo& g = cx.g;
  const Pos q = cell_pos<TX, TY, TZ>(p, cx.tg, cx.tile);
  double v[kNP];
#pragma unroll
  for (int s = 0; s < kNP; ++s) v[s] = 0.0;
  const double tf = g.cart ? 1.0 : g.tau;
  double R[14];
  const double cfl = tile_divergence<RT, TX, TY, TZ, true, false, VISC ? 2 : 0>(f.e1, f.u1, f.pi, p,
                                                                          eos, tf, q, R, lds);
  v[P_CFL] = cfl * p.h;
  double K[4] = {1.0, 0.0, 0.0, 0.0}, prev = 0.0;
  if (q.active) {
    const int c = q.c;
    const double e1 = f.e1[c], u1 = f.u1[0][c], u2 = f.u1[1][c], u3 = f.u1[2][c];
    double pc[10];
#pragma unroll
    for (int m = 0; m < 10; ++m) pc[m] = VISC ? f.pi[m][c] : 0.0;
    if (!g.cart) {
      double P, cs2;
      eos_p_cs2(eos, e1, P, cs2);
      const double w = (e1 > 0.0 ? e1 : 0.0) + P;
      const double ut = utau(u1, u2, u3);
      const double see = -(w * u3 * u3 + P + pc[9]);
      R[0] += see;
      R[3] += -(w * ut * u3 + pc[3]);
      v[P_GEO] = see;
    }
    double Tn[4];
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
      const double t0 = f.T[nu][c];
      Tn[nu] = t0 + 0.5 * ((f.T1[nu][c] - t0) + p.h * R[nu]);
      f.T[nu][c] = Tn[nu];
    }
    const double inv_tf1 = 1.0 / (g.cart ? 1.0 : g.tau1);
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) K[nu] = Tn[nu] * inv_tf1 - pc[nu];
    prev = e1;
    v[P_TSUM] = Tn[0];
  }
  const double x0 = root_guess<NET>(p, q.active, K[0], K[1], K[2], K[3], prev);
  if (q.active) {
    const int c = q.c;
    int it, fl;
    const Prim s = con2prim(eos, p, K[0], K[1], K[2], K[3], x0, it, fl);
    count_solve(v, it, fl);
    f.e[c] = s.e;
    f.up[0][c] = s.u1;  // becomes u~^{n+1} after the host swaps u and up
    f.up[1][c] = s.u2;
    f.up[2][c] = s.u3;
    v[P_EMAX] = s.e;
    v[P_VAC] = s.e == 0.0 ? 1.0 : 0.0;
  }
  block_partials(v, f.partial + (size_t)kNP * cx.tg.ntiles, cx.tg.ntiles, cx.tile);
}

// Folds the partials of stage1 and stage2T into the accumulated diagnostics.
// One workgroup per slot; each folds the slot's partials in a fixed order.
// acc: 0 geo_src, 1 max_cfl, 2 solves, 3 iter_sum, 4 iter_max, 5 fallbacks,
//      6 nonconv, 7 nans, 8 clamps, 9 eps_max, 10 sum_Ttt, 11 vacuum.
__global__ __launch_bounds__(kBlock) void k_reduce(const EventDesc* __restrict__ evs) {
  __shared__ double sh[2][kBlock / 64];
  const int e = blockIdx.x / kNP, s = blockIdx.x % kNP;
  const EventDesc& E = evs[e];
  const int nblk = E.tg.ntiles;
  const double* part = E.f.partial;
  const bool mx = is_max_slot(s);
  double x = 0.0, y = 0.0;  // stage1, stage2T
  for (int b = threadIdx.x; b < nblk; b += kBlock) {
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
  for (int w = 1; w < kBlock / 64; ++w) {
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

// pi~ as seen by readers: zero in vacuum cells.
__global__ __launch_bounds__(kBlock) void k_read_pi(const double* __restrict__ e,
                                                    const double* __restrict__ pi, double* dst,
                                                    int n) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c < n) dst[c] = e[c] == 0.0 ? 0.0 : pi[c];
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
  const double K0 = f.T[0][c] / tf - (pv ? f.pi[0][c] : 0.0);
  const double K1 = f.T[1][c] / tf - (pv ? f.pi[1][c] : 0.0);
  const double K2 = f.T[2][c] / tf - (pv ? f.pi[2][c] : 0.0);
  const double K3 = f.T[3][c] / tf - (pv ? f.pi[3][c] : 0.0);
  E[c] = K0;
  M[c] = sqrt(K1 * K1 + K2 * K2 + K3 * K3);
  eps[c] = e;
}

__global__ void k_zero(double* p, int n) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c < n) p[c] = 0.0;
}

// ---------------------------------------------------------------------------
// Tile shapes available to the launcher (the autotuner picks among them).
// ---------------------------------------------------------------------------
struct TileShape {
  int tx, ty, tz;
};
constexpr TileShape kTiles[] = {{4, 4, 16}, {2, 8, 16}, {4, 8, 8}, {1, 8, 32}, {16, 16, 1}, {256, 1, 1}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

}  // namespace ktmi

// ===========================================================================
// Host side: handle, workspace layout and the C ABI.
// ===========================================================================
using namespace ktmi;

enum { K_INIT = 0, K_FIRST, K_STAGE1, K_STAGE2PI, K_STAGE2T, K_REDUCE, K_COUNT };
static const char* kKernelNames[K_COUNT] = {"init", "first_estimate", "stage1", "stage2_pi",
                                            "stage2_T", "reduce"};

struct ktmi_handle {
  ktmi_desc d;
  std::string err;
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
  if ((double)d->nx * d->ny * d->ne > 2.0e9) {
    *why = "grid too large (more than 2e9 cells)";
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

static const int kNumFields = 39;  // e, u(3), up(3), pi(10), T(4), e1, u1(3), pi1(10), T1(4)

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
  p.inv_taupi_coef = h->d.etas > 0 ? 1.0 / (5.0 * h->d.etas * kHbarc) : 0.0;
  p.c_vac = sqrt(h->cs2_vac);
  p.eps_cut = h->d.eps_cut;
  p.theta = h->d.theta;
  p.newton_tol = h->d.newton_tol;
  p.pi_reg = h->d.pi_reg;
  p.newton_maxit = h->d.newton_maxit;
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

// One grouped launch of stencil kernel K over the events of a table that share
// a tile shape, precision and mode.
template <template <typename, int, int, int, bool> class K>
static void launch_class(hipStream_t s, int tile, int precision, bool net, const EventDesc* evs,
                         const GroupTable& gt) {
  const dim3 grid(gt.start[gt.nev]), block(kBlock);
  const bool mixed = precision == KTMI_MIXED;
  switch (tile) {
#define KTMI_TILE_CASE(id, X, Y, Z)                                  \
  case id:                                                           \
    if (mixed && net)                                                \
      K<float, X, Y, Z, true>::launch(grid, block, s, evs, gt);      \
    else if (mixed)                                                  \
      K<float, X, Y, Z, false>::launch(grid, block, s, evs, gt);     \
    else if (net)                                                    \
      K<double, X, Y, Z, true>::launch(grid, block, s, evs, gt);     \
    else                                                             \
      K<double, X, Y, Z, false>::launch(grid, block, s, evs, gt);    \
    break;
    KTMI_TILE_CASE(0, 4, 4, 16)
    KTMI_TILE_CASE(1, 2, 8, 16)
    KTMI_TILE_CASE(2, 4, 8, 8)
    KTMI_TILE_CASE(3, 1, 8, 32)
    KTMI_TILE_CASE(4, 16, 16, 1)
    KTMI_TILE_CASE(5, 256, 1, 1)
#undef KTMI_TILE_CASE
    default: break;
  }
}

// N: the kernel instance with the learned guess (only where a root solve
// takes a network guess; the others ignore it and are never launched with it).
#define KTMI_LAUNCHER(NAME, KERNEL)                                                       \
  template <typename RT, int X, int Y, int Z, bool N>                                     \
  struct NAME {                                                                           \
    static void launch(dim3 g, dim3 b, hipStream_t s, const EventDesc* evs, GroupTable gt) { \
      hipLaunchKernelGGL((KERNEL), g, b, 0, s, evs, gt);                                  \
    }                                                                                     \
  };
KTMI_LAUNCHER(LFirst, (k_first_estimate<RT, X, Y, Z>))
KTMI_LAUNCHER(LStage1V, (k_stage1<RT, X, Y, Z, true, N>))
KTMI_LAUNCHER(LStage1I, (k_stage1<RT, X, Y, Z, false, N>))
KTMI_LAUNCHER(LStage2Pi, (k_stage2_pi<RT, X, Y, Z>))
KTMI_LAUNCHER(LStage2TV, (k_stage2_T<RT, X, Y, Z, true, N>))
KTMI_LAUNCHER(LStage2TI, (k_stage2_T<RT, X, Y, Z, false, N>))
#undef KTMI_LAUNCHER

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
static int enqueue_class_step(ktmi_handle* h, hipStream_t s, int tile, int precision, int viscous,
                              bool net, const EventDesc* evs, const GroupTable& gt) {
  int rc;
  if (viscous) {
    rc = launch(h, K_STAGE1, [&] { launch_class<LStage1V>(s, tile, precision, net, evs, gt); });
    if (rc) return rc;
    rc = launch(h, K_STAGE2PI,
                [&] { launch_class<LStage2Pi>(s, tile, precision, false, evs, gt); });
    if (rc) return rc;
    return launch(h, K_STAGE2T,
                  [&] { launch_class<LStage2TV>(s, tile, precision, net, evs, gt); });
  }
  rc = launch(h, K_STAGE1, [&] { launch_class<LStage1I>(s, tile, precision, net, evs, gt); });
  if (rc) return rc;
  return launch(h, K_STAGE2T, [&] { launch_class<LStage2TI>(s, tile, precision, net, evs, gt); });
}

static bool uses_net(const ktmi_handle* h) { return h->d.guess == KTMI_GUESS_MLP; }

static int enqueue_step(ktmi_handle* h) {
  const GroupTable gt = single_table(h);
  int rc = enqueue_class_step(h, h->stream, h->tile, h->d.precision, h->d.viscous, uses_net(h),
                              h->dev_ev, gt);
  if (rc) return rc;
  return launch(h, K_REDUCE, [&] {
    hipLaunchKernelGGL(k_reduce, dim3(kNP), dim3(kBlock), 0, h->stream, h->dev_ev);
  });
}

static int finish_initial(ktmi_handle* h) {
  if (int rc = upload_event(h)) return rc;
  hipLaunchKernelGGL(k_set_clock, dim3(1), dim3(64), 0, h->stream, h->clock, h->tau);
  const GroupTable gt = single_table(h);
  int rc = launch(h, K_FIRST, [&] {
    launch_class<LFirst>(h->stream, h->tile, h->d.precision, false, h->dev_ev, gt);
  });
  if (rc) return rc;
  rc = launch(h, K_INIT, [&] {
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlock), 0, h->stream, h->f.acc, 32);
  });
  if (rc) return rc;
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
    int tile, precision, viscous;
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
    int rc = enqueue_class_step(h, g->stream, c.tile, c.precision, c.viscous, c.net, g->dev + c.first,
                                c.gt);
    if (rc) return group_fail(g, rc, h->err);
  }
  const int nev = (int)g->hs.size();
  hipLaunchKernelGGL(k_reduce, dim3(kNP * nev), dim3(kBlock), 0, g->stream, g->dev);
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
  d->pi_reg = 1.0;
  d->precision = KTMI_FP64;
  d->guess = KTMI_GUESS_PREV;
  d->tile = -1;
}

size_t ktmi_workspace_bytes(const ktmi_desc* d) {
  std::string why;
  if (!desc_ok(d, &why)) return 0;
  const size_t fs = field_stride(d);
  const size_t nb = (size_t)max_tiles(d);
  size_t bytes = (size_t)kNumFields * fs * sizeof(double);
  bytes += ((2 * nb * kNP + 31) / 32 * 32) * sizeof(double);  // partials
  bytes += 32 * sizeof(double);                               // accumulators
  bytes += 3 * (size_t)kEosMaxRows * sizeof(double);          // EoS table
  bytes += 3 * (size_t)kEosMaxRows * sizeof(float);           // its FP32 copy
  bytes += 4096 + 512;                                         // event table, clock
  bytes += (kMlpDevBytes + 255) / 256 * 256;                   // network parameters
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
  f.e = base + fs * q++;
  for (int m = 0; m < 3; ++m) f.u[m] = base + fs * q++;
  for (int m = 0; m < 3; ++m) f.up[m] = base + fs * q++;
  for (int m = 0; m < 10; ++m) f.pi[m] = base + fs * q++;
  for (int m = 0; m < 4; ++m) f.T[m] = base + fs * q++;
  f.e1 = base + fs * q++;
  for (int m = 0; m < 3; ++m) f.u1[m] = base + fs * q++;
  for (int m = 0; m < 10; ++m) f.pi1[m] = base + fs * q++;
  for (int m = 0; m < 4; ++m) f.T1[m] = base + fs * q++;
  double* rest = base + fs * q;
  f.partial = rest;
  rest += (2 * (size_t)max_tiles(&h->d) * kNP + 31) / 32 * 32;
  f.acc = rest;
  rest += 32;
  h->eos_store = rest;
  rest += 3 * (size_t)kEosMaxRows;                       // FP64 table
  rest += (3 * (size_t)kEosMaxRows * sizeof(float) + 7) / 8;  // FP32 copy
  rest = (double*)(((uintptr_t)rest + 255) / 256 * 256);
  h->dev_ev = (EventDesc*)rest;
  h->clock = rest + 4096 / 8;
  h->mlp_dev = (float*)(rest + (4096 + 512) / 8);
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
  h->eos.P = dP;
  h->eos.T = dT;
  h->eos.cs2 = dC;
  h->eos_set = true;
  h->ev_dirty = true;
  return KTMI_OK;
}

int ktmi_set_initial_primitive(ktmi_handle* h, const double* e, const double* ux,
                               const double* uy, const double* ue, const double* pi10) {
  if (!h) return KTMI_EINVAL;
  if (int rc = check_setup(h)) return rc;
  if (!e || !ux || !uy || !ue) return fail(h, KTMI_EINVAL, "null field pointer");
  const size_t n = (size_t)h->d.nx * h->d.ny * h->d.ne, nb = n * sizeof(double);
  hipStream_t s = h->stream;
  HIP_TRY(h, hipMemcpyAsync(h->f.e, e, nb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(h->f.u[0], ux, nb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(h->f.u[1], uy, nb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(h, hipMemcpyAsync(h->f.u[2], ue, nb, hipMemcpyDeviceToDevice, s));
  for (int m = 0; m < 10; ++m) {
    if (pi10 && h->d.viscous)
      HIP_TRY(h, hipMemcpyAsync(h->f.pi[m], pi10 + (size_t)m * n, nb, hipMemcpyDeviceToDevice, s));
    else
      hipLaunchKernelGGL(k_zero, dim3(h->nblk), dim3(kBlock), 0, s, h->f.pi[m], (int)n);
  }
  h->tau = h->d.tau0;
  const StepParams p = step_params(h);
  const Geo g = geo(h, h->tau, h->tau);
  int rc = launch(h, K_INIT, [&] {
    hipLaunchKernelGGL(k_init_primitive, dim3(h->nblk), dim3(kBlock), 0, s, h->f, p, h->eos, g,
                       h->d.viscous);
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
  for (int m = 0; m < 10; ++m) {
    if (pi10 && h->d.viscous)
      HIP_TRY(h, hipMemcpyAsync(h->f.pi[m], pi10 + (size_t)m * n, nb, hipMemcpyDeviceToDevice, s));
    else
      hipLaunchKernelGGL(k_zero, dim3(h->nblk), dim3(kBlock), 0, s, h->f.pi[m], (int)n);
  }
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
                       h->f.pi[field - KTMI_F_PI], dst, n);
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
  return KTMI_OK;
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
          g->classes[k].viscous == h->d.viscous && g->classes[k].net == uses_net(h))
        c = (int)k;
    if (c < 0) {
      ktmi_group::Class cl{};
      cl.tile = h->tile;
      cl.precision = h->d.precision;
      cl.viscous = h->d.viscous;
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
