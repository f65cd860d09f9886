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

namespace ktmi {

constexpr int kBlock = 256;
constexpr int kNP = 12;            // diagnostic partials per workgroup
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

// Tile grid of one launch.
struct TileGrid {
  int ntx, nty, ntz, ntiles;
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Workgroups are dispatched to the 8 XCDs round robin (block b -> XCD b % 8).
// Give XCD x a contiguous range of tile ids so neighbouring tiles share its L2.
__device__ __forceinline__ int tile_of_block(int nb) {
  const int b = blockIdx.x, x = b & 7, k = b >> 3;
  const int per = nb >> 3, rem = nb & 7;
  return x * per + (x < rem ? x : rem) + k;
}

// Position of this thread's cell.
struct Pos {
  int i, j, k;     // global cell coordinates
  int lx, ly, lz;  // coordinates inside the tile
  int i0, j0, k0;  // tile origin
  int c;           // flat index (valid only if active)
  bool active;
};

template <int TX, int TY, int TZ>
__device__ __forceinline__ Pos cell_pos(const StepParams& p, const TileGrid& tg) {
  Pos q;
  const int t = tile_of_block(tg.ntiles);
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
template <bool DO_T, bool DO_PI, int PI_SRC>
__device__ __forceinline__ double face_flux(const double* __restrict__ e, const double* const* u,
                                            const double* const* pi, int base, int a, int n,
                                            int stride, int axis, double tauf,
                                            const StepParams& p, const EosDev& eos,
                                            double H[14]) {
  int idx[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) idx[t] = base + clampi(a - 1 + t, 0, n - 1) * stride;
  double q4[14][4];
#pragma unroll
  for (int t = 0; t < 4; ++t) q4[0][t] = e[idx[t]];
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int t = 0; t < 4; ++t) q4[1 + m][t] = u[m][idx[t]];
#pragma unroll
  for (int m = 0; m < 10; ++m)
#pragma unroll
    for (int t = 0; t < 4; ++t) q4[4 + m][t] = ld_pi<PI_SRC>(pi, m, idx[t], q4[0][t]);
  bool vac = true;
  const int nchk = (PI_SRC == 2) ? 14 : 4;  // with PI_SRC 0/1, e == 0 implies pi~ = 0
#pragma unroll
  for (int v = 0; v < 14; ++v)
    if (v < nchk)
#pragma unroll
      for (int t = 0; t < 4; ++t) vac = vac && (q4[v][t] == 0.0);
  if (vac) {
#pragma unroll
    for (int k = 0; k < 14; ++k) H[k] = 0.0;
    return p.c_vac;
  }
  double qL[14], qR[14];
#pragma unroll
  for (int v = 0; v < 14; ++v) {
    qL[v] = q4[v][1] + 0.5 * mm_slope(p.theta, q4[v][0], q4[v][1], q4[v][2]);
    qR[v] = q4[v][2] - 0.5 * mm_slope(p.theta, q4[v][1], q4[v][2], q4[v][3]);
  }
  double QL[14], FL[14], QR[14], FR[14], sL, sR;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const double* q = side ? qR : qL;
    double* Q = side ? QR : QL;
    double* F = side ? FR : FL;
    const double ux = q[1], uy = q[2], ue = q[3];
    const double ut = sqrt(1.0 + ux * ux + uy * uy + ue * ue);
    double P, cs2;
    eos_p_cs2(eos, q[0], P, cs2);
    const double w = (q[0] > 0.0 ? q[0] : 0.0) + P;
    const double u4[4] = {ut, ux, uy, ue};
    const double ud = u4[axis];
    if (DO_T) {
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) {
        Q[nu] = tauf * (w * ut * u4[nu] - (nu == 0 ? P : 0.0) + q[4 + sym(0, nu)]);
        F[nu] = tauf * (w * ud * u4[nu] + (nu == axis ? P : 0.0) + q[4 + sym(axis, nu)]);
      }
    }
    if (DO_PI) {
#pragma unroll
      for (int m = 0; m < 10; ++m) {
        Q[4 + m] = ut * q[4 + m];
        F[4 + m] = ud * q[4 + m];
      }
    }
    const double s = local_speed(ut, ux, uy, ue, ud, cs2);
    if (side)
      sR = s;
    else
      sL = s;
  }
  const double c = fmax(sL, sR);
#pragma unroll
  for (int k = 0; k < 14; ++k) {
    const bool on = k < 4 ? DO_T : DO_PI;
    H[k] = on ? 0.5 * (FL[k] + FR[k]) - 0.5 * c * (QR[k] - QL[k]) : 0.0;
  }
  return c;
}

// KT flux divergence of the thread's cell over all three axes (Sec. III, eq. kt):
// R[q] = -sum_d (H_{+1/2} - H_{-1/2}) / Delta_d.  Every face of the tile is
// computed once by one thread and staged in LDS (component-major).  Returns
// max over the computed faces of c / Delta (for the CFL diagnostic).
template <int TX, int TY, int TZ, bool DO_T, bool DO_PI, int PI_SRC>
__device__ __forceinline__ double tile_divergence(const double* __restrict__ e,
                                                  const double* const* u, const double* const* pi,
                                                  const StepParams& p, const EosDev& eos,
                                                  double tauf, const Pos& q, double R[14],
                                                  double* lds) {
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
      double H[14];
      if (inrow && ga <= nd) {
        const int base = d == 0 ? (gj * p.ne + gk)
                                : (d == 1 ? (gi * p.ny) * p.ne + gk : (gi * p.ny + gj) * p.ne);
        const double c = face_flux<DO_T, DO_PI, PI_SRC>(e, u, pi, base, ga - 1, nd, stride, d + 1,
                                                        tauf, p, eos, H);
        cfl = fmax(cfl, c * inv_del);
      } else {
#pragma unroll
        for (int k = 0; k < 14; ++k) H[k] = 0.0;
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
#pragma unroll
      for (int k = 0; k < 14; ++k) R[k] -= (lds[k * F + fp] - lds[k * F + fm]) * inv_del;
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
__device__ __forceinline__ void pi_source(const double* const* u, const double* const* uE,
                                          const double* const* uL, const StepParams& p,
                                          const EosDev& eos, const Geo& g, const Pos& q,
                                          double ec, const double pc[10], double S[10]) {
  const int c0 = q.c;
  const int cart = g.cart;
  const double tau = g.tau;
  const double inv_tau = 1.0 / tau;
  const double uc[4] = {utau(u[0][c0], u[1][c0], u[2][c0]), u[0][c0], u[1][c0], u[2][c0]};
  double G[4][4];
  {
    const double a1 = uE[0][c0], a2 = uE[1][c0], a3 = uE[2][c0];
    const double b1 = uL[0][c0], b2 = uL[1][c0], b3 = uL[2][c0];
    const double ea[4] = {utau(a1, a2, a3), a1, a2, a3};
    const double eb[4] = {utau(b1, b2, b3), b1, b2, b3};
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) G[0][nu] = (eb[nu] - ea[nu]) * p.inv_h;
  }
  const int n3[3] = {p.nx, p.ny, p.ne};
  const int co[3] = {q.i, q.j, q.k};
  const int st[3] = {p.ny * p.ne, p.ne, 1};
  const double ihalf[3] = {0.5 * p.inv_dx, 0.5 * p.inv_dy, 0.5 * p.inv_de * (cart ? 1.0 : inv_tau)};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ip = c0 + (clampi(co[d] + 1, 0, n3[d] - 1) - co[d]) * st[d];
    const int im = c0 + (clampi(co[d] - 1, 0, n3[d] - 1) - co[d]) * st[d];
    const double p1 = u[0][ip], p2 = u[1][ip], p3 = u[2][ip];
    const double m1 = u[0][im], m2 = u[1][im], m3 = u[2][im];
    const double up4[4] = {utau(p1, p2, p3), p1, p2, p3};
    const double um4[4] = {utau(m1, m2, m3), m1, m2, m3};
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) G[d + 1][nu] = (up4[nu] - um4[nu]) * ihalf[d];
  }
  if (!cart) {
    G[3][0] += uc[3] * inv_tau;
    G[3][3] += uc[0] * inv_tau;
  }
  const double theta = G[0][0] + G[1][1] + G[2][2] + G[3][3];
  double a[4];
#pragma unroll
  for (int nu = 0; nu < 4; ++nu)
    a[nu] = uc[0] * G[0][nu] + uc[1] * G[1][nu] + uc[2] * G[2][nu] + uc[3] * G[3][nu];
  const double gt[4] = {1.0, -1.0, -1.0, -1.0};
  double b[4];
#pragma unroll
  for (int nu = 0; nu < 4; ++nu)
    b[nu] = pc[sym(nu, 0)] * a[0] - pc[sym(nu, 1)] * a[1] - pc[sym(nu, 2)] * a[2] -
            pc[sym(nu, 3)] * a[3];
  double P, T;
  eos_p_t(eos, ec, P, T);
  const double inv_taupi = T * p.inv_taupi_coef;
  const double eta_over_taupi = 0.2 * (ec + P);
  const double ue = uc[3];
  const double third = 1.0 / 3.0;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
    for (int nu = mu; nu < 4; ++nu) {
      const int m = sym(mu, nu);
      const double gmn = (mu == nu) ? gt[mu] : 0.0;
      const double sig = gt[mu] * G[mu][nu] + gt[nu] * G[nu][mu] - uc[mu] * a[nu] -
                         uc[nu] * a[mu] - 2.0 * third * (gmn - uc[mu] * uc[nu]) * theta;
      double s = -pc[m] * inv_taupi + eta_over_taupi * sig - pc[m] * theta * third -
                 (uc[mu] * b[nu] + uc[nu] * b[mu]);
      if (!cart) {
        double I = 0.0;  // Christoffel terms I^{mu nu}
        if (m == 0 || m == 9) I = 2.0 * ue * pc[3];
        else if (m == 1) I = ue * pc[6];
        else if (m == 2) I = ue * pc[8];
        else if (m == 3) I = ue * (pc[0] + pc[9]);
        else if (m == 6) I = ue * pc[1];
        else if (m == 8) I = ue * pc[2];
        s += -(pc[m] * uc[0] + I) * inv_tau;
      }
      S[m] = s;
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
__device__ __forceinline__ void block_partials(double v[kNP], double* out) {
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
    out[(size_t)s * gridDim.x + blockIdx.x] = x;  // slot-major: the reduce reads coalesced
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
__global__ __launch_bounds__(kBlock) void k_init_conserved(Fields f, StepParams p, EosDev eos,
                                                            Geo g, int visc) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= p.ncell) return;
  const double tf = g.cart ? 1.0 : g.tau;
  double pv[10];
#pragma unroll
  for (int m = 0; m < 10; ++m) pv[m] = visc ? f.pi[m][c] : 0.0;
  const double K0 = f.T[0][c] / tf - pv[0], K1 = f.T[1][c] / tf - pv[1];
  const double K2 = f.T[2][c] / tf - pv[2], K3 = f.T[3][c] / tf - pv[3];
  int it, fl;
  const Prim s = con2prim(eos, p, K0, K1, K2, K3, K0, it, fl);
  f.e[c] = s.e;
  f.u[0][c] = s.u1;
  f.u[1][c] = s.u2;
  f.u[2][c] = s.u3;
  if (s.e == 0.0 || !visc)
#pragma unroll
    for (int m = 0; m < 10; ++m) f.pi[m][c] = 0.0;
}

// First step: u*1 from one ideal forward-Euler step; u~^{-1} = 2 u~^0 - u*1.
template <int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_first_estimate(Fields f, StepParams p, EosDev eos,
                                                            Geo g, TileGrid tg) {
  __shared__ double lds[lds_doubles<TX, TY, TZ>()];
  const Pos q = cell_pos<TX, TY, TZ>(p, tg);
  const double tf = g.cart ? 1.0 : g.tau;
  double R[14];
  tile_divergence<TX, TY, TZ, true, false, 0>(f.e, f.u, f.pi, p, eos, tf, q, R, lds);
  if (!q.active) return;
  const int c = q.c;
  const double e = f.e[c], u1 = f.u[0][c], u2 = f.u[1][c], u3 = f.u[2][c];
  const double ut = utau(u1, u2, u3);
  double P, cs2;
  eos_p_cs2(eos, e, P, cs2);
  const double w = (e > 0.0 ? e : 0.0) + P;
  if (!g.cart) {
    R[0] += -(w * u3 * u3 + P);
    R[3] += -(w * ut * u3);
  }
  const double u4[4] = {ut, u1, u2, u3};
  double K[4];
  const double inv_tf1 = 1.0 / (g.cart ? 1.0 : g.tau1);
#pragma unroll
  for (int nu = 0; nu < 4; ++nu)
    K[nu] = (tf * (w * ut * u4[nu] - (nu == 0 ? P : 0.0)) + p.h * R[nu]) * inv_tf1;
  int it, fl;
  const Prim s = con2prim(eos, p, K[0], K[1], K[2], K[3], e, it, fl);
  f.up[0][c] = 2.0 * u1 - s.u1;
  f.up[1][c] = 2.0 * u2 - s.u2;
  f.up[2][c] = 2.0 * u3 - s.u3;
}

// Stage 1 at tau_n (predictor) for the ideal (VISC = false) or viscous path.
template <int TX, int TY, int TZ, bool VISC>
__global__ __launch_bounds__(kBlock) void k_stage1(Fields f, StepParams p, EosDev eos, Geo g,
                                                    TileGrid tg) {
  __shared__ double lds[lds_doubles<TX, TY, TZ>()];
  const Pos q = cell_pos<TX, TY, TZ>(p, tg);
  double v[kNP];
#pragma unroll
  for (int s = 0; s < kNP; ++s) v[s] = 0.0;
  const double tf = g.cart ? 1.0 : g.tau;
  double R[14];
  const double cfl =
      tile_divergence<TX, TY, TZ, true, VISC, VISC ? 1 : 0>(f.e, f.u, f.pi, p, eos, tf, q, R, lds);
  v[P_CFL] = cfl * p.h;
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
        pi_source(f.u, f.up, f.u, p, eos, g, q, e, pc, S);
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
    const double K0 = T1[0] * inv_tf1 - p1[0];
    int it, fl;
    const Prim s = con2prim(eos, p, K0, T1[1] * inv_tf1 - p1[1], T1[2] * inv_tf1 - p1[2],
                            T1[3] * inv_tf1 - p1[3], p.guess_cold ? K0 : e, it, fl);
    count_solve(v, it, fl);
    f.e1[c] = s.e;
    f.u1[0][c] = s.u1;
    f.u1[1][c] = s.u2;
    f.u1[2][c] = s.u3;
  }
  block_partials(v, f.partial);
}

// Stage 2, part 1 (tau_{n+1}): pi^{n+1} = [ (u^n pi^n + u* pi')/2 + h/2 R_pi(e', u', pi') ] / u'^tau.
template <int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_stage2_pi(Fields f, StepParams p, EosDev eos, Geo g,
                                                      TileGrid tg) {
  __shared__ double lds[lds_doubles<TX, TY, TZ>()];
  const Pos q = cell_pos<TX, TY, TZ>(p, tg);
  const double tf = g.cart ? 1.0 : g.tau;
  double R[14];
  tile_divergence<TX, TY, TZ, false, true, 2>(f.e1, f.u1, f.pi1, p, eos, tf, q, R, lds);
  if (!q.active) return;
  const int c = q.c;
  const double e1 = f.e1[c];
  double pc[10];
#pragma unroll
  for (int m = 0; m < 10; ++m) pc[m] = f.pi1[m][c];
  if (e1 >= p.eps_cut) {
    double S[10];
    pi_source(f.u1, f.u, f.u1, p, eos, g, q, e1, pc, S);
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
template <int TX, int TY, int TZ, bool VISC>
__global__ __launch_bounds__(kBlock) void k_stage2_T(Fields f, StepParams p, EosDev eos, Geo g,
                                                     TileGrid tg) {
  __shared__ double lds[lds_doubles<TX, TY, TZ>()];
  const Pos q = cell_pos<TX, TY, TZ>(p, tg);
  double v[kNP];
#pragma unroll
  for (int s = 0; s < kNP; ++s) v[s] = 0.0;
  const double tf = g.cart ? 1.0 : g.tau;
  double R[14];
  const double cfl = tile_divergence<TX, TY, TZ, true, false, VISC ? 2 : 0>(f.e1, f.u1, f.pi, p,
                                                                          eos, tf, q, R, lds);
  v[P_CFL] = cfl * p.h;
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
    const double K0 = Tn[0] * inv_tf1 - pc[0];
    int it, fl;
    const Prim s = con2prim(eos, p, K0, Tn[1] * inv_tf1 - pc[1], Tn[2] * inv_tf1 - pc[2],
                            Tn[3] * inv_tf1 - pc[3], p.guess_cold ? K0 : e1, it, fl);
    count_solve(v, it, fl);
    f.e[c] = s.e;
    f.up[0][c] = s.u1;  // becomes u~^{n+1} after the host swaps u and up
    f.up[1][c] = s.u2;
    f.up[2][c] = s.u3;
    v[P_EMAX] = s.e;
    v[P_TSUM] = Tn[0];
    v[P_VAC] = s.e == 0.0 ? 1.0 : 0.0;
  }
  block_partials(v, f.partial + (size_t)gridDim.x * kNP);
}

// Folds the partials of stage1 and stage2T into the accumulated diagnostics.
// One workgroup per slot; each folds the slot's partials in a fixed order.
// acc: 0 geo_src, 1 max_cfl, 2 solves, 3 iter_sum, 4 iter_max, 5 fallbacks,
//      6 nonconv, 7 nans, 8 clamps, 9 eps_max, 10 sum_Ttt, 11 vacuum.
__global__ __launch_bounds__(kBlock) void k_reduce(Fields f, int nblk, double half_h_vol,
                                                   double vol) {
  __shared__ double sh[2][kBlock / 64];
  const int s = blockIdx.x;
  const bool mx = is_max_slot(s);
  double x = 0.0, y = 0.0;  // stage1, stage2T
  for (int b = threadIdx.x; b < nblk; b += kBlock) {
    const double a = f.partial[(size_t)s * nblk + b];
    const double c = f.partial[(size_t)(kNP + s) * nblk + b];
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
  double* acc = f.acc;
  switch (s) {
    case P_GEO: acc[0] += half_h_vol * (x + y); break;
    case P_CFL: acc[1] = fmax(acc[1], fmax(x, y)); break;
    case P_EMAX: acc[9] = y; break;
    case P_TSUM: acc[10] = y * vol; break;
    case P_VAC: acc[11] = y; break;
    case P_ITMAX: acc[4] = fmax(acc[4], fmax(x, y)); break;
    default: acc[s] += x + y; break;
  }
}

// pi~ as seen by readers: zero in vacuum cells.
__global__ __launch_bounds__(kBlock) void k_read_pi(const double* __restrict__ e,
                                                    const double* __restrict__ pi, double* dst,
                                                    int n) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c < n) dst[c] = e[c] == 0.0 ? 0.0 : pi[c];
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
  if (d->precision != KTMI_FP64) {
    *why = "only KTMI_FP64 is available";
    return false;
  }
  if (d->guess != KTMI_GUESS_PREV && d->guess != KTMI_GUESS_COLD) {
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
  p.guess_cold = h->d.guess == KTMI_GUESS_COLD;
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

// Launches one stencil kernel family member for the handle's tile shape.
template <template <int, int, int> class K, typename... Args>
static void launch_tiled(const ktmi_handle* h, Args... args) {
  const dim3 grid(h->tg.ntiles), block(kBlock);
  switch (h->tile) {
#define KTMI_TILE_CASE(id, X, Y, Z) \
  case id: K<X, Y, Z>::launch(grid, block, h->stream, args...); break;
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

template <int X, int Y, int Z>
struct LFirst {
  static void launch(dim3 g, dim3 b, hipStream_t s, Fields f, StepParams p, EosDev e, Geo geo,
                     TileGrid tg) {
    hipLaunchKernelGGL((k_first_estimate<X, Y, Z>), g, b, 0, s, f, p, e, geo, tg);
  }
};
template <int X, int Y, int Z>
struct LStage1V {
  static void launch(dim3 g, dim3 b, hipStream_t s, Fields f, StepParams p, EosDev e, Geo geo,
                     TileGrid tg) {
    hipLaunchKernelGGL((k_stage1<X, Y, Z, true>), g, b, 0, s, f, p, e, geo, tg);
  }
};
template <int X, int Y, int Z>
struct LStage1I {
  static void launch(dim3 g, dim3 b, hipStream_t s, Fields f, StepParams p, EosDev e, Geo geo,
                     TileGrid tg) {
    hipLaunchKernelGGL((k_stage1<X, Y, Z, false>), g, b, 0, s, f, p, e, geo, tg);
  }
};
template <int X, int Y, int Z>
struct LStage2Pi {
  static void launch(dim3 g, dim3 b, hipStream_t s, Fields f, StepParams p, EosDev e, Geo geo,
                     TileGrid tg) {
    hipLaunchKernelGGL((k_stage2_pi<X, Y, Z>), g, b, 0, s, f, p, e, geo, tg);
  }
};
template <int X, int Y, int Z>
struct LStage2TV {
  static void launch(dim3 g, dim3 b, hipStream_t s, Fields f, StepParams p, EosDev e, Geo geo,
                     TileGrid tg) {
    hipLaunchKernelGGL((k_stage2_T<X, Y, Z, true>), g, b, 0, s, f, p, e, geo, tg);
  }
};
template <int X, int Y, int Z>
struct LStage2TI {
  static void launch(dim3 g, dim3 b, hipStream_t s, Fields f, StepParams p, EosDev e, Geo geo,
                     TileGrid tg) {
    hipLaunchKernelGGL((k_stage2_T<X, Y, Z, false>), g, b, 0, s, f, p, e, geo, tg);
  }
};

static int finish_initial(ktmi_handle* h) {
  const StepParams p = step_params(h);
  const int nb = h->nblk;
  const Geo g = geo(h, h->tau, h->tau + h->d.h);
  (void)nb;
  int rc = launch(h, K_FIRST, [&] { launch_tiled<LFirst>(h, h->f, p, h->eos, g, h->tg); });
  if (rc) return rc;
  rc = launch(h, K_INIT, [&] {
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(kBlock), 0, h->stream, h->f.acc, 32);
  });
  if (rc) return rc;
  h->step = 0;
  h->ready = true;
  return KTMI_OK;
}

static int check_setup(ktmi_handle* h) {
  if (!h->bound) return fail(h, KTMI_ESTATE, "no workspace bound");
  if (!h->eos_set) return fail(h, KTMI_ESTATE, "EoS table must be set after binding");
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
  h->bound = true;
  return KTMI_OK;
}

int ktmi_set_eos_conformal(ktmi_handle* h, double c_sb) {
  if (!h) return KTMI_EINVAL;
  if (!(c_sb > 0)) return fail(h, KTMI_EINVAL, "c_sb must be > 0");
  h->eos.kind = 0;
  h->eos.c_sb = c_sb;
  h->eos.inv_csb = 1.0 / c_sb;
  h->cs2_vac = 1.0 / 3.0;
  h->eos_set = true;
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
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->eos.kind = 1;
  h->eos.n = n;
  h->eos.e0 = e0;
  h->eos.de = de;
  h->eos.inv_de = 1.0 / de;
  h->cs2_vac = (e0 >= 0.0) ? cs2[0] : cs2[0];  // lookups clamp e = 0 to the first row
  h->eos.P = dP;
  h->eos.T = dT;
  h->eos.cs2 = dC;
  h->eos_set = true;
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
    hipLaunchKernelGGL(k_init_conserved, dim3(h->nblk), dim3(kBlock), 0, s, h->f, p, h->eos, g,
                       h->d.viscous);
  });
  if (rc) return rc;
  return finish_initial(h);
}

int ktmi_step(ktmi_handle* h, int nsteps) {
  if (!h) return KTMI_EINVAL;
  if (!h->ready) return fail(h, KTMI_ESTATE, "set an initial state first");
  if (nsteps < 0) return fail(h, KTMI_EINVAL, "negative step count");
  const StepParams p = step_params(h);
  hipStream_t s = h->stream;
  const double vol = h->d.dx * h->d.dy * h->d.de;
  for (int it = 0; it < nsteps; ++it) {
    const double t0 = h->tau, t1 = h->tau + h->d.h;
    const Geo g0 = geo(h, t0, t1), g1 = geo(h, t1, t1);
    const TileGrid tg = h->tg;
    int rc;
    if (h->d.viscous) {
      rc = launch(h, K_STAGE1, [&] { launch_tiled<LStage1V>(h, h->f, p, h->eos, g0, tg); });
      if (rc) return rc;
      rc = launch(h, K_STAGE2PI, [&] { launch_tiled<LStage2Pi>(h, h->f, p, h->eos, g1, tg); });
      if (rc) return rc;
      rc = launch(h, K_STAGE2T, [&] { launch_tiled<LStage2TV>(h, h->f, p, h->eos, g1, tg); });
    } else {
      rc = launch(h, K_STAGE1, [&] { launch_tiled<LStage1I>(h, h->f, p, h->eos, g0, tg); });
      if (rc) return rc;
      rc = launch(h, K_STAGE2T, [&] { launch_tiled<LStage2TI>(h, h->f, p, h->eos, g1, tg); });
    }
    if (rc) return rc;
    const int nt = tg.ntiles;
    rc = launch(h, K_REDUCE, [&] {
      hipLaunchKernelGGL(k_reduce, dim3(kNP), dim3(kBlock), 0, s, h->f, nt, 0.5 * h->d.h * vol,
                         vol);
    });
    if (rc) return rc;
    for (int m = 0; m < 3; ++m) std::swap(h->f.u[m], h->f.up[m]);
    h->tau = t1;
    h->step++;
  }
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
    src = h->f.u[field - KTMI_F_UX];
  else if (field >= KTMI_F_PI && field < KTMI_F_PI + 10) {
    hipLaunchKernelGGL(k_read_pi, dim3(h->nblk), dim3(kBlock), 0, s, h->f.e,
                       h->f.pi[field - KTMI_F_PI], dst, n);
    HIP_TRY(h, hipGetLastError());
    return KTMI_OK;
  } else if (field >= KTMI_F_T && field < KTMI_F_T + 4)
    src = h->f.T[field - KTMI_F_T];
  else if (field >= KTMI_F_UPREV && field < KTMI_F_UPREV + 3)
    src = h->f.up[field - KTMI_F_UPREV];
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
  return KTMI_OK;
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
  delete h;
}

}  // extern "C"
