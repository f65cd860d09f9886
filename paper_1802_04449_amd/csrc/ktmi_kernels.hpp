// ktmi_kernels.hpp -- gfx950 kernels of one RK2 step of the Kurganov-Tadmor
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
// L2).  Each pass writes per-workgroup diagnostic partials; the reduce kernel
// folds them in a fixed order, so results are bitwise reproducible.
//
// Template kernels only: the stencil passes are instantiated per (pass,
// arithmetic type) in ktmi_stencil.hip objects, the rest in ktmi.hip.
#pragma once
#ifndef KTMI_PI1_SPARSE
#define KTMI_PI1_SPARSE 1
#endif
#ifndef KTMI_S2PI_STREAM
#define KTMI_S2PI_STREAM 1
#endif
#include <hip/hip_runtime.h>

#include <math.h>

#include "../../include/ktmi.h"
#include "ktmi_device.hpp"
#include "ktmi_mlp.hpp"

namespace ktmi {

constexpr int kBlock = 256;
constexpr int kNP = 13;            // diagnostic partials per workgroup

constexpr int kEosMaxRows = 8192;  // table capacity reserved in the workspace

// Partial slots.  Sums: 0, 2, 3, 5-8, 10-12.  Maxima: 1, 4, 9.
enum : int {
  P_GEO = 0, P_CFL = 1, P_SOLVES = 2, P_ITSUM = 3, P_ITMAX = 4, P_FALLBACK = 5,
  P_NONCONV = 6, P_NAN = 7, P_CLAMP = 8, P_EMAX = 9, P_TSUM = 10, P_VAC = 11, P_NEG = 12
};
__host__ __device__ constexpr bool is_max_slot(int s) {
  return s == P_CFL || s == P_ITMAX || s == P_EMAX;
}

// Field pointers as the host fills them.  The fields of the state live in one
// workspace with a common stride; the pi~ block (and the stage-1 pi~ block)
// holds NQ consecutive fields: pi~ (0..9), then Pi (10) and n (11) with
// bulk/baryon.
struct Fields {
  double* e;       // e^n, overwritten by e^{n+1} in stage2T
  double* u[3];    // u~^n
  double* up[3];   // u~^{n-1}; stage2T writes u~^{n+1} here
  double* pi[12];  // pi~^n (0..9), then Pi (10) and n (11) with bulk/baryon (else null);
                   // overwritten by their n+1 values in stage2pi
  double* T[4];    // T~^{tau mu, n}, overwritten by T^{n+1} in stage2T
  double* e1;      // stage-1 prediction
  double* u1[3];
  double* pi1[12];
  double* T1[4];
  double* partial;  // [2][kNP][nblk]: stage1 then stage2T, slot-major
  double* acc;      // [16] accumulated diagnostics
  int* quiet;       // [4][ntiles]: quiet flags by clock parity (2), stage-2pi part (1),
                    // stage 1 T~' = T~^n (1)
  long fstride;     // elements from one field to the next
  int pf32;         // the pi~ blocks (pi, pi1) hold FP32 values (mixed precision)
};

// One field seen through the global address space.  Element i is addressed by
// a 32-bit byte offset from the field's base (fields hold fewer than 2^29
// elements; the host checks the grid size).
struct GField {
  gdouble* p;
  __device__ __forceinline__ double operator[](int i) const {
    return *(const gdouble*)((const gchar*)p + (unsigned)i * 8u);
  }
  __device__ __forceinline__ gdouble* operator+(int i) const {
    return (gdouble*)((gchar*)p + (unsigned)i * 8u);
  }
};

// The pi~ blocks (pi~, Pi, n and their stage-1 values) as stored: FP64, or FP32
// on the mixed-precision path (RT = float), element i of field k then at
// (float*)(base of field k) + i, in the first half of the field's slot.
template <typename RT>
__device__ __forceinline__ double ldq(const GField& g, int i) {
  if constexpr (sizeof(RT) == 4)
    return (double)*(const gfloat*)((const gchar*)g.p + (unsigned)i * 4u);
  else
    return g[i];
}
template <typename RT>
__device__ __forceinline__ void stq(const GField& g, int i, double v) {
  if constexpr (sizeof(RT) == 4)
    *(gfloat*)((gchar*)g.p + (unsigned)i * 4u) = (float)v;
  else
    *(g + i) = v;
}
// The same with the storage type chosen at run time (Fields::pf32), for the
// kernels that set up the state.
__device__ __forceinline__ double ldq_rt(const double* b, int i, int f32) {
  return f32 ? (double)((const float*)b)[i] : b[i];
}
__device__ __forceinline__ void stq_rt(double* b, int i, double v, int f32) {
  if (f32)
    ((float*)b)[i] = (float)v;
  else
    b[i] = v;
}

// Consecutive fields of one stride, seen through the global address space.
// The kernels hold one base pointer per group of fields instead of one per
// field: forty pointers held at once exceeded the scalar register file, and the
// compiler kept the spilled pointers in vector-register lanes, reloading them
// with v_readlane inside the face loops.
struct FSet {
  gdouble* b;  // first field of the group
  long fs;     // elements from one field to the next
  __device__ __forceinline__ GField operator[](int k) const { return GField{b + (long)k * fs}; }
};

struct DFields {
  GField e;
  FSet u, up, pi, T;
  GField e1;
  FSet u1, pi1, T1;
  gdouble* partial;
  gdouble* acc;
  gint* quiet;
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
  DFields f;
  StepParams p;
  EosDev eos;
  TileGrid tg;
  Geo g;
  int tile;  // tile index inside the event
  const gint* qcur;  // quiet flags after the previous step
  gint* qnext;       // quiet flags after this step
  gint* qpi;         // this step's stage-2pi part of the flags
  gint* t1same;      // this step's stage-1 flags: the tile's T~' equals T~^n (not stored)
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Store of a per-cell result of a stage pass.  Plain (cached) stores: the next
// pass reads these values, and non-temporal stores made the step 4% slower.
__device__ __forceinline__ void st_cell(gdouble* p, double v) { *p = v; }

// Workgroups are dispatched to the 8 XCDs round robin (block b -> XCD b % 8).
// Tiles are dealt to the XCDs in chunks of KTMI_CHUNK consecutive tile ids
// (chunk j -> XCD j % 8): inside a chunk consecutive tiles (eta, then y
// neighbours) share one XCD's L2, and every XCD gets chunks from all over the
// grid, so a grid whose matter sits in the middle (most heavy-ion events) loads
// the XCDs evenly.  The last nb % (8 KTMI_CHUNK) tiles map one to one.
#ifndef KTMI_CHUNK
#define KTMI_CHUNK 64
#endif
__device__ __forceinline__ int tile_of_block(int nb) {
  const int b = blockIdx.x, x = b & 7, k = b >> 3;
#if KTMI_CHUNK > 0
  constexpr int C = KTMI_CHUNK;
  const int K0 = (nb / (8 * C)) * C;  // blocks per XCD inside whole rounds of chunks
  if (k < K0) return ((k / C) * 8 + x) * C + k % C;
  return b;
#else
  // contiguous range of tile ids per XCD
  const int per = nb >> 3, rem = nb & 7;
  return x * per + (x < rem ? x : rem) + k;
#endif
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
  const long fs = E.f.fstride;
  c.f.e = GField{(gdouble*)E.f.e};
  c.f.pi = FSet{(gdouble*)E.f.pi[0], fs};
  c.f.T = FSet{(gdouble*)E.f.T[0], fs};
  c.f.e1 = GField{(gdouble*)E.f.e1};
  c.f.u1 = FSet{(gdouble*)E.f.u1[0], fs};
  c.f.pi1 = FSet{(gdouble*)E.f.pi1[0], fs};
  c.f.T1 = FSet{(gdouble*)E.f.T1[0], fs};
  c.f.partial = (gdouble*)E.f.partial;
  c.f.acc = (gdouble*)E.f.acc;
  c.f.quiet = (gint*)E.f.quiet;
  c.p = E.p;
  c.eos = E.eos;
  c.tg = E.tg;
  const double tau = E.clock[0];
  const bool odd = E.clock[2] != 0.0;
  c.f.u = FSet{(gdouble*)(odd ? E.f.up[0] : E.f.u[0]), fs};
  c.f.up = FSet{(gdouble*)(odd ? E.f.u[0] : E.f.up[0]), fs};
  c.g.cart = E.cart;
  c.g.tau1 = tau + E.p.h;
  c.g.tau = stage2 ? c.g.tau1 : tau;
  c.tile = t - gt.start[e];
  const int nt = E.tg.ntiles;
  c.qcur = c.f.quiet + (odd ? nt : 0);
  c.qnext = c.f.quiet + (odd ? 0 : nt);
  c.qpi = c.f.quiet + 2 * nt;
  c.t1same = c.f.quiet + 3 * nt;
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

// Quiet tiles (optional, StepParams::quiet_r[0] > 0).  A tile is quiet after a
// step when every cell had e = 0 before the step, after stage 1 and after it,
// pi~ = 0 after stage 1 and after it, and K^tau below the cutoff: its state is
// a vacuum with at most a dilute T~ that no flux or source changes.  A step can
// skip a tile (no loads, no stores) when every tile within quiet_r tiles
// (6 cells: the reach of stage 1 and stage 2 stencils and gradients) was
// quiet after the previous step: all three passes would then reproduce exactly
// the values its buffers hold.  Returns the block-uniform decision.
template <int TX, int TY, int TZ>
__device__ __forceinline__ bool tile_asleep(const StepParams& p, const TileGrid& tg,
                                            const gint* __restrict__ qcur, int tile) {
  if (p.quiet_r[0] <= 0) return false;
  const int tk = tile % tg.ntz, r = tile / tg.ntz;
  const int tj = r % tg.nty, ti = r / tg.nty;
  const int rx = p.quiet_r[0], ry = p.quiet_r[1], rz = p.quiet_r[2];
  const int wx = 2 * rx + 1, wy = 2 * ry + 1, wz = 2 * rz + 1;
  int awake = 0;
  for (int n = threadIdx.x; n < wx * wy * wz; n += kBlock) {
    const int a = ti - rx + n / (wy * wz), b = tj - ry + (n / wz) % wy, c = tk - rz + n % wz;
    if (a < 0 || a >= tg.ntx || b < 0 || b >= tg.nty || c < 0 || c >= tg.ntz) continue;
    awake |= qcur[(a * tg.nty + b) * tg.ntz + c] == 0;
  }
  return __syncthreads_or(awake) == 0;
}

// Max over the tile's faces of c / Delta when every face is a vacuum face.
template <typename RT>
__device__ __forceinline__ double vacuum_cfl(const StepParams& p, double tauf) {
  const double cv = (double)(RT)p.c_vac;
  double cfl = 0.0;
  if (p.nx > 1) cfl = fmax(cfl, cv * p.inv_dx);
  if (p.ny > 1) cfl = fmax(cfl, cv * p.inv_dy);
  if (p.ne > 1) cfl = fmax(cfl, cv * (p.inv_de / tauf));
  return cfl;
}

// pi~ at a cell: PI_SRC 0 -> 0, 1 -> zero where e == 0 (vacuum), 2 -> as stored.
template <int PI_SRC, typename RT>
__device__ __forceinline__ double ld_pi(const FSet& pi, int m, int idx, double e) {
  if (PI_SRC == 0) return 0.0;
  const double v = ldq<RT>(pi[m], idx);
  if (PI_SRC == 1) return e == 0.0 ? 0.0 : v;
  return v;
}

// KT face flux H = [F(Q^r) + F(Q^l)]/2 - c (Q^r - Q^l)/2 (Sec. III, eq. flux_out)
// at the face between cells a and a+1 along `axis` (1 = x, 2 = y, 3 = eta),
// from a minmod reconstruction of the primitives on the 4-cell stencil
// a-1 .. a+2 (generalized minmod with theta; zero-gradient boundaries by index
// clamping).  Q_T = tau Tc^{tau nu}, F_T = tau Tc^{axis nu}; Q_pi = u~^tau
// pi~, F_pi = u~^axis pi~; c = max local speed of the two face states.  The
// components the pass uses (T~'s if DO_T, pi~'s if DO_PI) go to out[k * F];
// returns c.  BK: the transported set also holds the bulk pressure Pi (k = 14),
// which adds to P in T~'s Q and F (eqn. Pitilde), and the net-baryon density n
// (k = 15); both have the flux form of the pi~ components.
//
// Evaluated as a stream to keep few values live: e and u~ first (face states,
// u~^tau, P, c_s^2, e + P, speeds, the fluid part of T~'s Q and F), then one
// pi~ component at a time (its face states, its own flux, its terms in T~'s Q
// and F), then T~'s flux.  The arithmetic of every component is that of
// tau (w u u - P g + pi) and u pi as written, in that order.
template <typename R, bool DO_T, bool DO_PI, int PI_SRC, bool BK = false>
__device__ __forceinline__ R face_flux_stream(const GField& e, const FSet& u,
                                       const FSet& pi, int base, int a, int n,
                                       int stride, int axis, R tauf, const StepParams& p,
                                       const EosDev& eos, R* out, int F,
                                       GField ez = GField{nullptr}) {
  int idx[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) idx[t] = base + clampi(a - 1 + t, 0, n - 1) * stride;
  constexpr int NQ = BK ? 12 : 10;
  // Vacuum faces: every state the kernels write has u~ = 0 where e = 0, and
  // pi~ reads as zero there (PI_SRC 0/1; as stored in stage 2T, whose pi^{n+1}
  // the regulator zeroed wherever e' is zero), so e alone decides and a vacuum
  // face skips the other loads.
  double ev[4];
  bool vac = true;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    ev[t] = e[idx[t]];
    vac = vac && (ev[t] == 0.0);
  }
  // As-stored pi~ (PI_SRC 2) is zero wherever the energy density it was
  // regulated with is zero when the regulator zeroes it there (vac_zero): the
  // pass's own e (stage 2T), or ez (stage 2pi: e^n), then also tested here;
  // without vac_zero such a face is evaluated in full.
  // SPARSE: stage 1 leaves pi~' unstored where e^n = 0 (vac_zero), so stage 2pi
  // reads it masked by e^n (ez), as stage 1 masks pi~^n by e^n
  constexpr bool SPARSE = KTMI_PI1_SPARSE && PI_SRC == 2 && !BK;
  const bool zmask = SPARSE && ez.p != nullptr && p.vac_zero;
  double ezv[4] = {1.0, 1.0, 1.0, 1.0};
  if (zmask) {
#pragma unroll
    for (int t = 0; t < 4; ++t) ezv[t] = ez[idx[t]];
  }
  if (PI_SRC == 2 && vac && ez.p != nullptr && p.vac_zero) {
#pragma unroll
    for (int t = 0; t < 4; ++t) vac = vac && (zmask ? ezv[t] : ez[idx[t]]) == 0.0;
  }
  if (vac && (PI_SRC != 2 || p.vac_zero)) {
#pragma unroll
    for (int k = 0; k < 4 + NQ; ++k)
      if (k < 4 ? DO_T : DO_PI) out[k * F] = R(0);
    return (R)p.c_vac;
  }
  const R th = (R)p.theta;
  // the pi~ components the face needs; the first one's loads go out with u~'s
  auto needed = [&](int m) {
    if (m == 10 || PI_SRC == 0) return false;  // Pi: with e and u~ below
    bool inT = false;
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) inT = inT || m == sym(0, nu) || m == sym(axis, nu);
    return DO_PI || (DO_T && inT);
  };
  auto next_needed = [&](int m) {
    int k = m + 1;
    while (k < NQ && !needed(k)) ++k;
    return k;
  };
  double pcur[4], pnext[4];
  // e and u~ face states (and Pi's, which T~'s pressure needs)
  constexpr int NV = BK ? 5 : 4;
  R fL[NV], fR[NV];
  {
    R q4[NV][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) q4[0][t] = (R)ev[t];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int t = 0; t < 4; ++t) q4[1 + m][t] = (R)u[m][idx[t]];
    {
      const int m0 = next_needed(-1);
      if (m0 < NQ) {
#pragma unroll
        for (int t = 0; t < 4; ++t) pcur[t] = ldq<R>(pi[m0], idx[t]);
      }
    }
    if constexpr (BK) {
#pragma unroll
      for (int t = 0; t < 4; ++t) q4[4][t] = (R)ld_pi<PI_SRC, R>(pi, 10, idx[t], ev[t]);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      fL[v] = q4[v][1] + R(0.5) * mm_slope_r<R>(th, q4[v][0], q4[v][1], q4[v][2]);
      fR[v] = q4[v][2] - R(0.5) * mm_slope_r<R>(th, q4[v][1], q4[v][2], q4[v][3]);
    }
  }
  R ut[2], ud[2], AQ[2][4], AF[2][4], sp[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const R* q = side ? fR : fL;
    const R ux = q[1], uy = q[2], ue = q[3];
    ut[side] = sqrt(R(1) + ux * ux + uy * uy + ue * ue);
    R P, cs2;
    eos_p_cs2_r<R>(eos, q[0], P, cs2);
    if constexpr (BK) P = P + q[4];  // P + Pi
    const R w = (q[0] > R(0) ? q[0] : R(0)) + P;
    const R u4[4] = {ut[side], ux, uy, ue};
    ud[side] = u4[axis];
    if (DO_T) {
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) {
        AQ[side][nu] = w * ut[side] * u4[nu] - (nu == 0 ? P : R(0));
        AF[side][nu] = w * ud[side] * u4[nu] + (nu == axis ? P : R(0));
      }
    }
    sp[side] = local_speed_r<R>(ut[side], ux, uy, ue, ud[side], cs2);
  }
  const R c = fmax(sp[0], sp[1]);
  if constexpr (BK) {
    if (DO_PI) {  // Pi's own flux
      const R QL = ut[0] * fL[4], QR = ut[1] * fR[4];
      const R FL = ud[0] * fL[4], FR = ud[1] * fR[4];
      out[14 * F] = R(0.5) * (FL + FR) - R(0.5) * c * (QR - QL);
    }
  }
  // pi~ components (and n), one at a time; the next needed component's loads
  // are issued before the current one is used, so one round trip to the cache
  // overlaps the arithmetic of the previous component
#pragma unroll
  for (int m = 0; m < NQ; ++m) {
    if (!needed(m)) {  // no pi~ (ideal), Pi, or a component T~'s flux does not use
      if (DO_PI && m != 10) out[(4 + m) * F] = R(0);
      continue;
    }
    const int mn = next_needed(m);
    if (mn < NQ) {
#pragma unroll
      for (int t = 0; t < 4; ++t) pnext[t] = ldq<R>(pi[mn], idx[t]);
    }
    R p4[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
      p4[t] = (R)((PI_SRC == 1 && ev[t] == 0.0) || (zmask && ezv[t] == 0.0) ? 0.0 : pcur[t]);
    const R pL = p4[1] + R(0.5) * mm_slope_r<R>(th, p4[0], p4[1], p4[2]);
    const R pR = p4[2] - R(0.5) * mm_slope_r<R>(th, p4[1], p4[2], p4[3]);
    if (DO_PI) {
      const R QL = ut[0] * pL, QR = ut[1] * pR;
      const R FL = ud[0] * pL, FR = ud[1] * pR;
      out[(4 + m) * F] = R(0.5) * (FL + FR) - R(0.5) * c * (QR - QL);
    }
    if (DO_T) {
#pragma unroll
      for (int nu = 0; nu < 4; ++nu) {
        if (m == sym(0, nu)) {
          AQ[0][nu] = AQ[0][nu] + pL;
          AQ[1][nu] = AQ[1][nu] + pR;
        }
        if (m == sym(axis, nu)) {
          AF[0][nu] = AF[0][nu] + pL;
          AF[1][nu] = AF[1][nu] + pR;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) pcur[t] = pnext[t];
  }
#pragma unroll
  for (int nu = 0; nu < 4; ++nu) {
    if (DO_T) {
      const R Q0 = tauf * AQ[0][nu], Q1 = tauf * AQ[1][nu];
      const R F0 = tauf * AF[0][nu], F1 = tauf * AF[1][nu];
      out[nu * F] = R(0.5) * (F0 + F1) - R(0.5) * c * (Q1 - Q0);
    }
  }
  return c;
}

// KT face flux H = [F(Q^r) + F(Q^l)]/2 - c (Q^r - Q^l)/2 (Sec. III, eq. flux_out)
// at the face between cells a and a+1 along `axis` (1 = x, 2 = y, 3 = eta).
// `base` is the flat index of the row's cell with coordinate 0 along the axis.
// Components 0..3: T~^{d nu} part (if DO_T); 4..13: u~^d pi~ part (if DO_PI);
// BK: 14, 15 the u~^d Pi and u~^d n parts (Pi also adds to P in T~'s part).
// Returns the face's local speed c.  A face whose four stencil cells are exact
// vacuum (all primitives zero) has H = 0 and c = c_vac, so it skips the arithmetic.
// R is the arithmetic type (double, or float on the mixed-precision path).
template <typename R, bool DO_T, bool DO_PI, int PI_SRC, bool BK = false>
__device__ __forceinline__ R face_flux_all(const GField& e, const FSet& u,
                                       const FSet& pi, int base, int a, int n,
                                       int stride, int axis, R tauf, const StepParams& p,
                                       const EosDev& eos, R* out, int F) {
  int idx[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) idx[t] = base + clampi(a - 1 + t, 0, n - 1) * stride;
  // Vacuum faces skip all arithmetic.  Every state the kernels write has u~ = 0
  // where e = 0 (the root solve and the cutoff return all-zero primitives), and
  // with PI_SRC 0/1 pi~ reads as zero there too, so e alone decides: it is
  // loaded first and a vacuum face skips the other loads.  As-stored pi~
  // (PI_SRC 2) can be nonzero where e = 0, so there the whole stencil is loaded
  // at once (no dependent second round of loads) and e and pi~ decide.
  constexpr int NQ = BK ? 12 : 10, NC = 4 + NQ;
  double ev[4];
  bool vac = true;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    ev[t] = e[idx[t]];
    vac = vac && (ev[t] == 0.0);
  }
  R q4[NC][4];
  if (PI_SRC == 2) {
    // Without the pi~ flux only the components in T~'s density (tau nu) and
    // flux (axis nu) matter (and Pi): the others are neither loaded nor tested.
#pragma unroll
    for (int m = 0; m < NQ; ++m) {
      const bool used = DO_PI || m < 4 || m == sym(axis, 1) || m == sym(axis, 2) ||
                        m == sym(axis, 3) || m == 10;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double x = used ? ldq<R>(pi[m], idx[t]) : 0.0;
        vac = vac && (x == 0.0);
        q4[4 + m][t] = (R)x;
      }
    }
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int t = 0; t < 4; ++t) q4[1 + m][t] = (R)u[m][idx[t]];
  }
  if (vac) {  // only the components the pass uses: the LDS holds no others
#pragma unroll
    for (int k = 0; k < NC; ++k)
      if (k < 4 ? DO_T : DO_PI) out[k * F] = R(0);
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
    for (int m = 0; m < NQ; ++m)
#pragma unroll
      for (int t = 0; t < 4; ++t) q4[4 + m][t] = (R)ld_pi<PI_SRC, R>(pi, m, idx[t], ev[t]);
  }
  R qL[NC], qR[NC];
  const R th = (R)p.theta;
#pragma unroll
  for (int v = 0; v < NC; ++v) {
    const R a0 = q4[v][0], a1 = q4[v][1], a2 = q4[v][2], a3 = q4[v][3];
    qL[v] = a1 + R(0.5) * mm_slope_r<R>(th, a0, a1, a2);
    qR[v] = a2 - R(0.5) * mm_slope_r<R>(th, a1, a2, a3);
  }
  // Scalars of the two states first (u~^tau, P, c_s^2, e + P, speed), then each
  // flux component from them and the face states, straight to LDS: only the
  // face states stay live, not the Q and F arrays of both sides.
  R ut[2], P[2], w[2], ud[2], sp[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const R* q = side ? qR : qL;
    const R ux = q[1], uy = q[2], ue = q[3];
    ut[side] = sqrt(R(1) + ux * ux + uy * uy + ue * ue);
    R cs2;
    eos_p_cs2_r<R>(eos, q[0], P[side], cs2);
    if constexpr (BK) P[side] = P[side] + q[14];  // P + Pi
    w[side] = (q[0] > R(0) ? q[0] : R(0)) + P[side];
    const R u4[4] = {ut[side], ux, uy, ue};
    ud[side] = u4[axis];
    sp[side] = local_speed_r<R>(ut[side], ux, uy, ue, ud[side], cs2);
  }
  const R c = fmax(sp[0], sp[1]);
  if (DO_T) {
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
      R Q[2], Fx[2];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const R* q = side ? qR : qL;
        const R un = nu == 0 ? ut[side] : q[nu];
        Q[side] = tauf * (w[side] * ut[side] * un - (nu == 0 ? P[side] : R(0)) + q[4 + sym(0, nu)]);
        Fx[side] =
            tauf * (w[side] * ud[side] * un + (nu == axis ? P[side] : R(0)) + q[4 + sym(axis, nu)]);
      }
      out[nu * F] = R(0.5) * (Fx[0] + Fx[1]) - R(0.5) * c * (Q[1] - Q[0]);
    }
  }
#pragma unroll
  for (int m = 0; m < NQ; ++m) {
    if (DO_PI) {
      const R QL = ut[0] * qL[4 + m], QR = ut[1] * qR[4 + m];
      const R FL = ud[0] * qL[4 + m], FR = ud[1] * qR[4 + m];
      out[(4 + m) * F] = R(0.5) * (FL + FR) - R(0.5) * c * (QR - QL);
    }
  }
  return c;
}

// Faces of a TX x TY x TZ tile along each axis, F_d = (T_d + 1) N / T_d, split
// into M_d = kBlock floor(F_d / kBlock) faces evaluated in full rounds (one face
// per thread and round) and R_d = F_d - M_d remainder faces.  The remainders of
// the three axes are evaluated together in one round (their own LDS area), so a
// 4x4x16 tile takes 4 rounds of face evaluations (144 remainder faces, then 256
// per axis) instead of 6 in which every axis' second round keeps one wave busy.
// Measured on the 201x201x105 grids this speeds up stage 1 by 5-13%; stage 2pi
// gains on a grid without vacuum but loses up to 30% on the hotspot grid, where
// most of its faces are vacuum faces loaded in full and rounds that mix axes cost
// more (also with a window of x and y faces that adds no code), so the layout is
// chosen per pass: SPLIT = false puts every face in full rounds (M_d = F_d, no
// remainder).
template <int TX, int TY, int TZ, bool SPLIT = true>
struct FaceLayout {
  static constexpr int N = TX * TY * TZ;
  static constexpr int F0 = (TX + 1) * (N / TX), F1 = (TY + 1) * (N / TY), F2 = (TZ + 1) * (N / TZ);
  static constexpr int M0 = SPLIT ? F0 / kBlock * kBlock : F0;
  static constexpr int M1 = SPLIT ? F1 / kBlock * kBlock : F1;
  static constexpr int M2 = SPLIT ? F2 / kBlock * kBlock : F2;
  static constexpr int R0 = F0 - M0, R1 = F1 - M1, R2 = F2 - M2;
  static constexpr int RSUM = R0 + R1 + R2;
  static constexpr int MMAX = M0 > M1 ? (M0 > M2 ? M0 : M2) : (M1 > M2 ? M1 : M2);
  static_assert(RSUM <= kBlock, "remainder faces must fit one round");
};

// Face f of axis d (0 x, 1 y, 2 eta) of the thread's tile: its flux components go
// to out[k * S] (zeros for a face outside the grid); returns c / Delta_d (0 outside).
template <typename RT, int TX, int TY, int TZ, bool DO_T, bool DO_PI, int PI_SRC, bool BK>
__device__ __forceinline__ double eval_face(const GField& e, const FSet& u,
                                            const FSet& pi, const StepParams& p,
                                            const EosDev& eos, double tauf, const Pos& q, int d,
                                            int f, RT* out, int S, GField ez = GField{nullptr}) {
  constexpr int NC = BK ? 16 : 14;
  const int nd = d == 0 ? p.nx : (d == 1 ? p.ny : p.ne);
  const double inv_del = d == 0 ? p.inv_dx : (d == 1 ? p.inv_dy : p.inv_de / tauf);
  const int stride = d == 0 ? p.ny * p.ne : (d == 1 ? p.ne : 1);
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
  if (inrow && ga <= nd) {
    const int base = d == 0 ? (gj * p.ne + gk)
                            : (d == 1 ? (gi * p.ny) * p.ne + gk : (gi * p.ny + gj) * p.ne);
    // stage 1 (pi~ masked by e): the streamed evaluation (fewer registers);
    // stage 2 (as-stored pi~): all loads at once with the per-face e/pi~ test
    RT c;
    if constexpr (PI_SRC == 2 && DO_PI && !KTMI_S2PI_STREAM)
      c = face_flux_all<RT, DO_T, DO_PI, PI_SRC, BK>(e, u, pi, base, ga - 1, nd, stride, d + 1,
                                                     (RT)tauf, p, eos, out, S);
    else
      c = face_flux_stream<RT, DO_T, DO_PI, PI_SRC, BK>(e, u, pi, base, ga - 1, nd, stride, d + 1,
                                                        (RT)tauf, p, eos, out, S, ez);
    return (double)c * inv_del;
  }
#pragma unroll
  for (int k = 0; k < NC; ++k)
    if (k < 4 ? DO_T : DO_PI) out[k * S] = RT(0);
  return 0.0;
}

// KT flux divergence of the thread's cell over all three axes (Sec. III, eq. kt):
// R[q] = -sum_d (H_{+1/2} - H_{-1/2}) / Delta_d.  Every face of the tile is
// computed once by one thread and staged in LDS (component-major).  Returns
// max over the computed faces of c / Delta (for the CFL diagnostic).  BK: R and
// the LDS hold 16 components (with Pi and n).  SPLIT: the face rounds of FaceLayout.
// ALLF (T~'s components only): the faces of all three axes in one sequence of
// rounds, F0 + F1 + F2 of them (912 for a 4x4x16 tile: 4 rounds instead of 6),
// with one barrier; their 4 components fit lds_doubles_allf (29 KB).
template <typename RT, int TX, int TY, int TZ, bool DO_T, bool DO_PI, int PI_SRC, bool BK = false,
          bool SPLIT = false, bool ALLF = false, bool ZERO_R = true>
__device__ __forceinline__ double tile_divergence(const GField& e,
                                                  const FSet& u, const FSet& pi,
                                                  const StepParams& p, const EosDev& eos,
                                                  double tauf, const Pos& q, double* R,
                                                  RT* lds, GField ez = GField{nullptr}) {
  constexpr int N = TX * TY * TZ;
  constexpr int NQ = BK ? 12 : 10, NC = 4 + NQ;
  if constexpr (ZERO_R) {
#pragma unroll
    for (int k = 0; k < NC; ++k) R[k] = 0.0;
  }
  double cfl = 0.0;
  const int tid = threadIdx.x;
  // Whole-tile vacuum test.  Every face stencil of the tile reads cells in the
  // box [i0 - 2, i0 + TX + 1] x [j0 - 2, j0 + TY + 1] x [k0 - 2, k0 + TZ + 1]
  // (clamped to the grid).  When that box is vacuum (e = 0, and in the stage-2
  // passes, whose faces read as-stored pi~, also pi~ = 0), every face is a vacuum
  // face: H = 0, c = c_vac, the values the per-face test gives, decided in one
  // or two rounds of loads for the whole workgroup instead of one per face
  // round.  In stage 1 (pi~ masked by e) it saves 4% of the pass on the
  // 201x201x105 hotspot grid and costs 1% on a grid without vacuum.
#ifndef KTMI_S1_TILE_TEST
#define KTMI_S1_TILE_TEST 1
#endif
  if (PI_SRC == 2 || KTMI_S1_TILE_TEST) {
    constexpr int BX = TX + 4, BY = TY + 4, BZ = TZ + 4, NB = BX * BY * BZ;
    // the tile's own cells first (one load per thread, which the cell phase
    // reuses): a tile with matter skips the rest of the test
    int nz = q.active && e[q.c] != 0.0;
    int any = __syncthreads_or(nz);
    if (!any) {
      for (int b = tid; b < NB; b += kBlock) {
        const int bx = b / (BY * BZ), by = (b / BZ) % BY, bz = b % BZ;
        const int i = clampi(q.i0 - 2 + bx, 0, p.nx - 1), j = clampi(q.j0 - 2 + by, 0, p.ny - 1);
        const int k = clampi(q.k0 - 2 + bz, 0, p.ne - 1);
        nz |= e[(i * p.ny + j) * p.ne + k] != 0.0;
      }
      any = __syncthreads_or(nz);
    }
    // e = 0 in the whole box: as-stored pi~ decides.  Where the regulator zeroes
    // pi~ with zero e (vac_zero), pi~ is zero wherever the energy density it was
    // regulated with is: the pass's own e (ez.p null: nothing more to test), or ez
    // (one field instead of the NQ components).
    if (PI_SRC == 2 && !any && !(p.vac_zero && ez.p == nullptr)) {
      for (int b = tid; b < NB; b += kBlock) {
        const int bx = b / (BY * BZ), by = (b / BZ) % BY, bz = b % BZ;
        const int i = clampi(q.i0 - 2 + bx, 0, p.nx - 1), j = clampi(q.j0 - 2 + by, 0, p.ny - 1);
        const int k = clampi(q.k0 - 2 + bz, 0, p.ne - 1);
        const int c = (i * p.ny + j) * p.ne + k;
        if (p.vac_zero) {
          nz |= ez[c] != 0.0;
        } else {
#pragma unroll
          for (int m = 0; m < NQ; ++m) nz |= ldq<RT>(pi[m], c) != 0.0;
        }
      }
      any = __syncthreads_or(nz);
    }
    if (!any) return vacuum_cfl<RT>(p, tauf);
  }
  if constexpr (ALLF) {
    static_assert(!DO_PI, "all faces at once hold T~'s components only");
    using L = FaceLayout<TX, TY, TZ, false>;
    constexpr int FT = L::F0 + L::F1 + L::F2;
    // (for the 4x4x16 tile the axis is uniform over each wave in every round)
    for (int g = tid; g < FT; g += kBlock) {
      if (g < L::F0) {
        if (p.nx > 1)
          cfl = fmax(cfl, eval_face<RT, TX, TY, TZ, DO_T, DO_PI, PI_SRC, BK>(
                              e, u, pi, p, eos, tauf, q, 0, g, lds + g, FT));
      } else if (g < L::F0 + L::F1) {
        if (p.ny > 1)
          cfl = fmax(cfl, eval_face<RT, TX, TY, TZ, DO_T, DO_PI, PI_SRC, BK>(
                              e, u, pi, p, eos, tauf, q, 1, g - L::F0, lds + g, FT));
      } else {
        if (p.ne > 1)
          cfl = fmax(cfl, eval_face<RT, TX, TY, TZ, DO_T, DO_PI, PI_SRC, BK>(
                              e, u, pi, p, eos, tauf, q, 2, g - L::F0 - L::F1, lds + g, FT));
      }
    }
    __syncthreads();
    if (q.active) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int nd = d == 0 ? p.nx : (d == 1 ? p.ny : p.ne);
        if (nd == 1) continue;  // both faces see identical states: zero divergence
        int fm, fp;
        if (d == 0) {
          fm = q.lx * (TY * TZ) + q.ly * TZ + q.lz;
          fp = fm + TY * TZ;
        } else if (d == 1) {
          fm = L::F0 + q.lx * ((TY + 1) * TZ) + q.ly * TZ + q.lz;
          fp = fm + TZ;
        } else {
          fm = L::F0 + L::F1 + (q.lx * TY + q.ly) * (TZ + 1) + q.lz;
          fp = fm + 1;
        }
        const RT rinv = (RT)(d == 0 ? p.inv_dx : (d == 1 ? p.inv_dy : p.inv_de / tauf));
#pragma unroll
        for (int k = 0; k < 4; ++k) R[k] -= (double)((lds[k * FT + fp] - lds[k * FT + fm]) * rinv);
      }
    }
    __syncthreads();
  } else if constexpr (SPLIT) {
    using L = FaceLayout<TX, TY, TZ, SPLIT>;
    RT* const rem = lds + NC * L::MMAX;  // remainder faces, axis after axis
    // Remainder round: the last R_d faces of every axis, one per thread.
    if constexpr (L::RSUM > 0) {
      if (tid < L::R0) {
        if (p.nx > 1)
          cfl = fmax(cfl, eval_face<RT, TX, TY, TZ, DO_T, DO_PI, PI_SRC, BK>(
                              e, u, pi, p, eos, tauf, q, 0, L::M0 + tid, rem + tid, L::R0));
      } else if (tid < L::R0 + L::R1) {
        const int t = tid - L::R0;
        if (p.ny > 1)
          cfl = fmax(cfl, eval_face<RT, TX, TY, TZ, DO_T, DO_PI, PI_SRC, BK>(
                              e, u, pi, p, eos, tauf, q, 1, L::M1 + t, rem + NC * L::R0 + t, L::R1));
      } else if (tid < L::RSUM) {
        const int t = tid - L::R0 - L::R1;
        if (p.ne > 1)
          cfl = fmax(cfl, eval_face<RT, TX, TY, TZ, DO_T, DO_PI, PI_SRC, BK>(
                              e, u, pi, p, eos, tauf, q, 2, L::M2 + t,
                              rem + NC * (L::R0 + L::R1) + t, L::R2));
      }
    }
  #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int nd = d == 0 ? p.nx : (d == 1 ? p.ny : p.ne);
      if (nd == 1) continue;  // both faces see identical states: zero divergence
      const int M = d == 0 ? L::M0 : (d == 1 ? L::M1 : L::M2);
      const int Rd = d == 0 ? L::R0 : (d == 1 ? L::R1 : L::R2);
      RT* const remd = rem + NC * (d == 0 ? 0 : (d == 1 ? L::R0 : L::R0 + L::R1));
      for (int f = tid; f < M; f += kBlock)
        cfl = fmax(cfl, eval_face<RT, TX, TY, TZ, DO_T, DO_PI, PI_SRC, BK>(e, u, pi, p, eos, tauf,
                                                                             q, d, f, lds + f, M));
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
        // slot of face f: the full-round area (stride M) or the remainder area (stride R_d)
        const bool mm = Rd == 0 || fm < M, mp = Rd == 0 || fp < M;
        const RT* const am = mm ? lds + fm : remd + (fm - M);
        const RT* const ap = mp ? lds + fp : remd + (fp - M);
        const int sm = mm ? M : Rd, sp = mp ? M : Rd;
        const RT rinv = (RT)(d == 0 ? p.inv_dx : (d == 1 ? p.inv_dy : p.inv_de / tauf));
  #pragma unroll
        for (int k = 0; k < NC; ++k)  // only the components this pass evaluates
          if (k < 4 ? DO_T : DO_PI) R[k] -= (double)((ap[k * sp] - am[k * sm]) * rinv);
      }
      __syncthreads();
    }
  } else {
  #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int nd = d == 0 ? p.nx : (d == 1 ? p.ny : p.ne);
      if (nd == 1) continue;  // both faces see identical states: zero divergence
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
        if (inrow && ga <= nd) {
          const int base = d == 0 ? (gj * p.ne + gk)
                                  : (d == 1 ? (gi * p.ny) * p.ne + gk : (gi * p.ny + gj) * p.ne);
          RT c;
          if constexpr (PI_SRC == 2 && DO_PI && !KTMI_S2PI_STREAM)
            c = face_flux_all<RT, DO_T, DO_PI, PI_SRC, BK>(e, u, pi, base, ga - 1, nd, stride, d + 1,
                                                           (RT)tauf, p, eos, lds + f, F);
          else
            c = face_flux_stream<RT, DO_T, DO_PI, PI_SRC, BK>(e, u, pi, base, ga - 1, nd, stride,
                                                              d + 1, (RT)tauf, p, eos, lds + f, F,
                                                              ez);
          cfl = fmax(cfl, (double)c * inv_del);
        } else {
  #pragma unroll
          for (int k = 0; k < NC; ++k)
            if (k < 4 ? DO_T : DO_PI) lds[k * F + f] = RT(0);
        }
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
        for (int k = 0; k < NC; ++k)  // only the components this pass evaluates
          if (k < 4 ? DO_T : DO_PI) R[k] -= (double)((lds[k * F + fp] - lds[k * F + fm]) * rinv);
      }
      __syncthreads();
    }
  }
  (void)N;
  return cfl;
}

// LDS elements of the face fluxes: NC components of the largest full-round
// face set plus the remainders of the three axes.
template <int TX, int TY, int TZ, int NC = 14, bool SPLIT = false>
constexpr int lds_doubles() {
  using L = FaceLayout<TX, TY, TZ, SPLIT>;
  return NC * (L::MMAX + L::RSUM);
}

// LDS elements of tile_divergence's ALLF layout: T~'s 4 components of every face.
template <int TX, int TY, int TZ>
constexpr int lds_doubles_allf() {
  using L = FaceLayout<TX, TY, TZ, false>;
  return 4 * (L::F0 + L::F1 + L::F2);
}

// Waves per SIMD asked of the stage-2 passes: at least 3 where the tile's LDS
// leaves room for three workgroups per CU (160 KB), else no bound.  The cap was
// a net gain when these passes needed more registers (stage2_pi 10-16%,
// stage2_T 1-5% on the 201x201x105 grids, with a few spilled registers; the
// lambda_1 variant 8% in FP64 with 60 bytes of spill, 13% in FP32); the plain
// stage2_pi now fits 123 VGPRs (FP64, four waves) and 91 (FP32, five) without
// it.  Stage1 loses from the cap, so it has none, nor has the bulk variant of
// stage2_pi (it spilled 96 bytes a lane under the cap: 1.06 ms against 0.75 ms
// without it; its stage2_T keeps the cap).  NOCAP = true asks for no bound.
template <typename RT, int TX, int TY, int TZ, bool NOCAP, int NC = 14>
constexpr int pi_waves() {
  return !NOCAP && 163840 / (int)(lds_doubles<TX, TY, TZ, NC>() * sizeof(RT) + 512) >= 3 ? 3 : 1;
}

// Waves per SIMD asked of stage 2T: four without bulk in FP64 (its streamed faces
// need 143 VGPRs; under the four-wave cap of 128 a few spill, and the pass still
// runs faster: 0.46 -> 0.42 ms on the 201x201x105 hotspot grid, 0.86 -> 0.84 ms
// on the grid without vacuum), five in FP32 (95 VGPRs, no spill: 0.36 -> 0.33 ms
// and 0.64 -> 0.60 ms); with bulk as the other stage-2 passes.
template <typename RT, int TX, int TY, int TZ, bool BK>
constexpr int s2t_waves() {
  return !BK ? (sizeof(RT) == 4 ? 5 : 4) : pi_waves<RT, TX, TY, TZ, false>();
}

// u~^tau of spatial components.
__device__ __forceinline__ double utau(double a, double b, double c) {
  return sqrt(1.0 + a * a + b * b + c * c);
}

// Israel-Stewart source (Sec. II, eqns. pitilde, Ipi; eqn. pimn with lambda_2 = lambda_3 = 0):
// S = -(pi - eta sigma)/tau_pi - pi theta/3 - (u b + b u) - pi u~^tau/tau - I
//     - (lambda_1/tau_pi) pi^<mu_l pi^nu>l,
// sigma~, theta, D~u~ from nabla~_mu u~^nu (eq. dtuz), b^nu = pi^{nu beta} g_{beta beta} a^beta.
// uE/uL: time levels for d_tau u~.  With eta = (eta/s)(e+P) hbarc/T and
// tau_pi = b (eta/s) hbarc/T (b = 5 in Sec. II), eta/tau_pi = (e+P)/b.  lambda_1 =
// lambda1_hat / e (Sec. V.C scaling); the bracket <> is the double projector of
// eqn. projector applied to X^{ab} = pi^{a l} g_{l l} pi^{b l}, expanded as
// X - u w - w u + u u (u.w) - (1/3)(g - u u)(g:X - u.w) with w^b = u_a X^{ab}
// (an identity for any symmetric X; pi's transversality is not assumed).
// BK adds the sources of Pi and n (eqns. Pitilde, Ntilde):
// S_Pi = -(Pi + zeta theta)/tau_Pi - Pi theta/3 - Pi u~^tau/tau (zeta / tau_Pi =
// (e + P)/c for tau_Pi = c (zeta/s) hbarc / T), S_n = -n u~^tau/tau; pc_d and
// S_d then hold 12 components.
template <typename R, bool L1, bool BK = false>
__device__ __forceinline__ void pi_source(const FSet& u, const FSet& uE,
                                          const FSet& uL, const StepParams& p,
                                          const EosDev& eos, const Geo& g, const Pos& q,
                                          double ec_d, const double* pc_d, double* S_d) {
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
  const R eta_over_taupi = (R)p.eta_taupi * (ec + P);
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
  if constexpr (BK) {
    const R Pi = (R)pc_d[10], nb = (R)pc_d[11];
    R sPi = -Pi * (T * (R)p.inv_taubulk_coef) - (R)p.zeta_taubulk * (ec + P) * theta -
            Pi * theta * third;
    R sn = R(0);
    if (!cart) {
      sPi -= Pi * uc[0] * inv_tau;
      sn = -(nb * uc[0] * inv_tau);
    }
    S_d[10] = p.bulk ? (double)sPi : 0.0;
    S_d[11] = p.baryon ? (double)sn : 0.0;
  }
  if constexpr (L1) {
    R X[10];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = a; b < 4; ++b)
        X[sym(a, b)] = pc[sym(a, 0)] * pc[sym(b, 0)] - pc[sym(a, 1)] * pc[sym(b, 1)] -
                       pc[sym(a, 2)] * pc[sym(b, 2)] - pc[sym(a, 3)] * pc[sym(b, 3)];
    R w[4];  // w^b = u_a X^{ab}, u_a = g_a u~^a
#pragma unroll
    for (int b = 0; b < 4; ++b)
      w[b] = uc[0] * X[sym(0, b)] - uc[1] * X[sym(1, b)] - uc[2] * X[sym(2, b)] -
             uc[3] * X[sym(3, b)];
    const R uw = uc[0] * w[0] - uc[1] * w[1] - uc[2] * w[2] - uc[3] * w[3];
    const R tr = X[0] - X[4] - X[7] - X[9] - uw;  // Delta_{ab} X^{ab}
    const R c1 = (R)p.lambda1_hat / ec * inv_taupi;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
#pragma unroll
      for (int nu = mu; nu < 4; ++nu) {
        const int m = sym(mu, nu);
        const R dmn = ((mu == nu) ? gt[mu] : R(0)) - uc[mu] * uc[nu];
        const R Y = X[m] - uc[mu] * w[nu] - uc[nu] * w[mu] + uc[mu] * uc[nu] * uw - third * dmn * tr;
        S_d[m] -= (double)(c1 * Y);
      }
    }
  }
}

// Scale pi~ so that sqrt(|pi~:pi~|) <= pi_reg (e+P); zero it where e+P = 0.
// BK: Pi is clipped to [-P, P] and Pi, n are zero where e+P = 0 too.
template <bool BK = false>
__device__ __forceinline__ void regulate(const EosDev& eos, const StepParams& p, double e,
                                         double* pv) {
  if (!(p.pi_reg > 0.0)) return;
  constexpr int NQ = BK ? 12 : 10;
  double P, c;
  eos_p_cs2(eos, e, P, c);
  const double w = (e > 0.0 ? e : 0.0) + P;
  if (!(w > 0.0)) {
#pragma unroll
    for (int m = 0; m < NQ; ++m) pv[m] = 0.0;
    return;
  }
  if constexpr (BK) pv[10] = fmin(fmax(pv[10], -P), P);
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
__device__ __forceinline__ void block_partials(double v[kNP], gdouble* out, int ntiles, int tile) {
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
  if (fl & kNeg) v[P_NEG] += 1.0;
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
    for (int m = 0; m < 10; ++m) pv[m] = visc ? f.pi1[m][c] : 0.0;  // staged FP64 input
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
#pragma unroll
  for (int m = 0; m < 10; ++m) stq_rt(f.pi[m], c, s.e == 0.0 || !visc ? 0.0 : pv[m], f.pf32);
}

// First step: u*1 from one ideal forward-Euler step; u~^{-1} = 2 u~^0 - u*1.
template <typename RT, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_first_estimate(const EventDesc* __restrict__ evs,
                                                            GroupTable gt) {
  __shared__ RT lds[lds_doubles<TX, TY, TZ>()];
  const Ctx cx = load_ctx(evs, gt, 0);
  const DFields& f = cx.f;
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
  st_cell(f.up[0] + c, 2.0 * u1 - s.u1);
  st_cell(f.up[1] + c, 2.0 * u2 - s.u2);
  st_cell(f.up[2] + c, 2.0 * u3 - s.u3);
}

// A cell's e, u~ and (VISC) pi~ at the current level; u~ and pi~ read as zero
// (no loads) where e = 0.
template <typename RT, bool VISC, int NQ>
__device__ __forceinline__ void cell_values(const DFields& f, int c, double& e, double& u1,
                                            double& u2, double& u3, double* pc) {
  e = f.e[c];
  u1 = u2 = u3 = 0.0;
#pragma unroll
  for (int m = 0; m < NQ; ++m) pc[m] = 0.0;
  if (e != 0.0) {
    u1 = f.u[0][c];
    u2 = f.u[1][c];
    u3 = f.u[2][c];
    if (VISC) {
#pragma unroll
      for (int m = 0; m < NQ; ++m) pc[m] = ldq<RT>(f.pi[m], c);
    }
  }
}

// Stage 1 at tau_n (predictor) for the ideal (VISC = false) or viscous path;
// BK (viscous only): also Pi and n, with P + Pi in T~ and in the root solve.
// The cell's sources come before the face rounds, so the shear source's
// gradients and the divergence accumulators are never live together: 137 VGPRs
// in FP64 (three waves per SIMD, which its 45 KB of LDS also allows; 161 with the
// sources after the rounds), 103 in FP32 (four waves; 134 before, and the pass
// went from 0.54 to 0.49 ms on the 201x201x105 hotspot grid), which asks for
// five (96 VGPRs with 14 spilled: 0.43 -> 0.41 ms there).  The bulk variant
// and the network variants ask for three waves (uncapped, the matrix-core
// results take 32 accumulation registers on top; capped, they stay in VGPRs
// without spills), the network variant with the lambda_1 term two (else one).
template <typename RT, int TX, int TY, int TZ, bool VISC, bool NET, bool L1, bool BK = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    BK || (NET && !L1) ? 3 : (NET ? 2 : (sizeof(RT) == 4 ? 5 : 1))))) void k_stage1(const EventDesc* __restrict__ evs,
                                                    GroupTable gt) {
  constexpr int NQ = BK ? 12 : 10;
  __shared__ RT lds[lds_doubles<TX, TY, TZ, 4 + NQ, true>()];
  const Ctx cx = load_ctx(evs, gt, 0);
  const DFields& f = cx.f;
  const StepParams& p = cx.p;
  const EosDev& eos = cx.eos;
  const Geo& g = cx.g;
  const Pos q = cell_pos<TX, TY, TZ>(p, cx.tg, cx.tile);
  double v[kNP];
#pragma unroll
  for (int s = 0; s < kNP; ++s) v[s] = 0.0;
  const double tf = g.cart ? 1.0 : g.tau;
  if (tile_asleep<TX, TY, TZ>(p, cx.tg, cx.qcur, cx.tile)) {
    v[P_CFL] = vacuum_cfl<RT>(p, tf) * p.h;  // what the vacuum faces would give
    // the stage-1 root solve of a quiet cell sees K^tau = T~^{tau tau}/tau_{n+1}
    if (q.active) v[P_NEG] = f.T[0][q.c] < 0.0 ? 1.0 : 0.0;
    block_partials(v, f.partial, cx.tg.ntiles, cx.tile);
    return;
  }
  double R[4 + NQ];
#pragma unroll
  for (int k = 0; k < 4 + NQ; ++k) R[k] = 0.0;
  // The cell's sources first (geometric, and the shear relaxation source with its
  // velocity gradients): their registers are free again before the face rounds
  // accumulate the flux divergence onto them.
  // e = 0 implies u~ = 0 (the cutoff and the root solve return zero velocity
  // with zero energy density), and pi~ reads as zero there: no loads
  if (q.active) {
    const int c = q.c;
    double e, u1, u2, u3, pc[NQ];
    cell_values<RT, VISC, NQ>(f, c, e, u1, u2, u3, pc);
    if (!g.cart) {  // geometric source S_T = (-Tc^{ee}, 0, 0, -Tc^{te})
      const double ut = utau(u1, u2, u3);
      double P, cs2;
      eos_p_cs2(eos, e, P, cs2);
      if constexpr (BK) P += pc[10];
      const double w = (e > 0.0 ? e : 0.0) + P;
      const double see = -(w * u3 * u3 + P + pc[9]);
      R[0] = see;
      R[3] = -(w * ut * u3 + pc[3]);
      v[P_GEO] = see;
    }
    if (VISC && e >= p.eps_cut) {
      double S[NQ];
      pi_source<RT, L1, BK>(f.u, f.up, f.u, p, eos, g, q, e, pc, S);
#pragma unroll
      for (int m = 0; m < NQ; ++m) R[4 + m] = S[m];
    }
  }
  const double cfl = tile_divergence<RT, TX, TY, TZ, true, VISC, VISC ? 1 : 0, BK, true, false,
                                     false>(f.e, f.u, f.pi, p, eos, tf, q, R, lds);
  v[P_CFL] = cfl * p.h;
  double K[4] = {1.0, 0.0, 0.0, 0.0}, prev = 0.0, Pi1 = 0.0;
  double T1[4];
  bool t1same = true;  // T~' = T~^n bitwise in this cell (no flux or source)
  if (q.active) {
    const int c = q.c;
    // the cell's values again (cache hits after the face rounds)
    double e, u1, u2, u3, pc[NQ];
    cell_values<RT, VISC, NQ>(f, c, e, u1, u2, u3, pc);
    const double ut = utau(u1, u2, u3);
    double p1[NQ];
    if (VISC) {
      // u* = 2u^n - u^{n-1}: not needed where pi~' is zero whatever it is
      bool zero = e == 0.0;
#pragma unroll
      for (int m = 0; m < NQ; ++m) zero = zero && R[4 + m] == 0.0;
      double inv_uts = 1.0;
      if (!zero) {
        const double s1 = 2.0 * u1 - f.up[0][c], s2 = 2.0 * u2 - f.up[1][c],
                     s3 = 2.0 * u3 - f.up[2][c];
        inv_uts = 1.0 / utau(s1, s2, s3);
      }
#pragma unroll
      for (int m = 0; m < NQ; ++m) p1[m] = (ut * pc[m] + p.h * R[4 + m]) * inv_uts;
      regulate<BK>(eos, p, e, p1);
      // with vac_zero, pi~' is zero where e^n is: stage 2pi reads it masked there
      if (!(KTMI_PI1_SPARSE && !BK && p.vac_zero && e == 0.0)) {
#pragma unroll
        for (int m = 0; m < NQ; ++m) stq<RT>(f.pi1[m], c, p1[m]);
      }
      if constexpr (BK) Pi1 = p1[10];
    } else {
#pragma unroll
      for (int m = 0; m < NQ; ++m) p1[m] = 0.0;
    }
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) {
      const double t0 = f.T[nu][c];
      T1[nu] = t0 + p.h * R[nu];
      t1same = t1same && __builtin_bit_cast(long long, T1[nu]) == __builtin_bit_cast(long long, t0);
    }
    const double inv_tf1 = 1.0 / (g.cart ? 1.0 : g.tau1);
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) K[nu] = T1[nu] * inv_tf1 - p1[nu];
    prev = e;
  }
  // A tile whose T~' equals T~^n in every cell (a vacuum tile: no flux, no
  // source) does not store it; stage 2T reads T~^n for it instead (the flag is
  // written every step, so no state carries over between steps).
  const int all_same = __syncthreads_and(t1same);
  if (!all_same && q.active) {
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) st_cell(f.T1[nu] + q.c, T1[nu]);
  }
  if (threadIdx.x == 0) cx.t1same[cx.tile] = all_same;
  const double x0 = root_guess<NET>(p, q.active, K[0], K[1], K[2], K[3], prev);
  if (q.active) {
    const int c = q.c;
    int it, fl;
    const Prim s = con2prim<BK>(eos, p, K[0], K[1], K[2], K[3], x0, it, fl, Pi1);
    count_solve(v, it, fl);
    st_cell(f.e1 + c, s.e);
    st_cell(f.u1[0] + c, s.u1);
    st_cell(f.u1[1] + c, s.u2);
    st_cell(f.u1[2] + c, s.u3);
  }
  block_partials(v, f.partial, cx.tg.ntiles, cx.tile);
}

// Stage 2, part 1 (tau_{n+1}): pi^{n+1} = [ (u^n pi^n + u* pi')/2 + h/2 R_pi(e', u', pi') ] / u'^tau.
// BK: Pi^{n+1} and n^{n+1} the same way.  The relaxation source comes before the
// face rounds: 123 VGPRs in FP64 (four waves per SIMD; 139 and three with the
// source after them: 0.45 -> 0.40 ms on the 201x201x105 hotspot grid, 1.04 ->
// 0.96 ms without vacuum), 91 in FP32 (five waves: 0.32 -> 0.30 ms).
template <typename RT, int TX, int TY, int TZ, bool L1, bool BK = false>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(pi_waves<RT, TX, TY, TZ, BK, BK ? 16 : 14>()))) void k_stage2_pi(
    const EventDesc* __restrict__ evs, GroupTable gt) {
  constexpr int NQ = BK ? 12 : 10;
  __shared__ RT lds[lds_doubles<TX, TY, TZ, 4 + NQ>()];
  const Ctx cx = load_ctx(evs, gt, 1);
  const DFields& f = cx.f;
  const StepParams& p = cx.p;
  const EosDev& eos = cx.eos;
  const Geo& g = cx.g;
  const Pos q = cell_pos<TX, TY, TZ>(p, cx.tg, cx.tile);
  if (tile_asleep<TX, TY, TZ>(p, cx.tg, cx.qcur, cx.tile)) return;
  const double tf = g.cart ? 1.0 : g.tau;
  double R[4 + NQ];
#pragma unroll
  for (int k = 0; k < 4 + NQ; ++k) R[k] = 0.0;
  // The cell's relaxation source first (as in stage 1: its gradients' registers
  // are free again before the face rounds accumulate the divergence onto it).
  // Where e' = 0 the regulator zeroes pi^{n+1} (vac_zero): no source needed.
  if (q.active) {
    const int c = q.c;
    const double e1 = f.e1[c];
    if (!(e1 == 0.0 && p.vac_zero) && e1 >= p.eps_cut) {
      double pc[NQ], S[NQ];
      const bool zm = KTMI_PI1_SPARSE && !BK && p.vac_zero && f.e[c] == 0.0;  // pi~' unstored
#pragma unroll
      for (int m = 0; m < NQ; ++m) pc[m] = zm ? 0.0 : ldq<RT>(f.pi1[m], c);
      pi_source<RT, L1, BK>(f.u1, f.u, f.u1, p, eos, g, q, e1, pc, S);
#pragma unroll
      for (int m = 0; m < NQ; ++m) R[4 + m] = S[m];
    }
  }
  // pi~' was regulated with e^n in stage 1: zero wherever e^n is (vac_zero)
  tile_divergence<RT, TX, TY, TZ, false, true, 2, BK, false, false, false>(
      f.e1, f.u1, f.pi1, p, eos, tf, q, R, lds, f.e);
  bool quiet = true;  // this cell's part of the quiet-tile test
  if (q.active) {
    const int c = q.c;
    const double e1 = f.e1[c];
    // where e' = 0 the regulator zeroes pi^{n+1} (vac_zero): nothing to load
    // unless the quiet-tile test needs this cell's pi~'
    const bool vz = e1 == 0.0 && p.vac_zero;
    double pc[NQ];
#pragma unroll
    for (int m = 0; m < NQ; ++m) pc[m] = 0.0;
    if ((!vz || p.quiet_r[0] > 0) &&
        !(KTMI_PI1_SPARSE && !BK && p.vac_zero && f.e[c] == 0.0)) {  // else unstored, zero
#pragma unroll
      for (int m = 0; m < NQ; ++m) pc[m] = ldq<RT>(f.pi1[m], c);
    }
    double pn[NQ];
#pragma unroll
    for (int m = 0; m < NQ; ++m) pn[m] = 0.0;
    double en = 0.0;
    if (!vz) {
      en = f.e[c];
      const double a1 = f.u[0][c], a2 = f.u[1][c], a3 = f.u[2][c];
      const double utn = utau(a1, a2, a3);
      const double uts = utau(2.0 * a1 - f.up[0][c], 2.0 * a2 - f.up[1][c], 2.0 * a3 - f.up[2][c]);
      const double inv_ut1 = 1.0 / utau(f.u1[0][c], f.u1[1][c], f.u1[2][c]);
      double pin[NQ];  // pi~^n, zero where e^n = 0
#pragma unroll
      for (int m = 0; m < NQ; ++m) pin[m] = 0.0;
      if (en != 0.0) {
#pragma unroll
        for (int m = 0; m < NQ; ++m) pin[m] = ldq<RT>(f.pi[m], c);
      }
#pragma unroll
      for (int m = 0; m < NQ; ++m)
        pn[m] = (0.5 * (utn * pin[m] + uts * pc[m]) + 0.5 * p.h * R[4 + m]) * inv_ut1;
      regulate<BK>(eos, p, e1, pn);
    } else if (p.quiet_r[0] > 0) {
      en = f.e[c];
    }
#pragma unroll
    for (int m = 0; m < NQ; ++m) stq<RT>(f.pi[m], c, pn[m]);
    quiet = en == 0.0 && e1 == 0.0;
#pragma unroll
    for (int m = 0; m < NQ; ++m) quiet = quiet && pc[m] == 0.0 && pn[m] == 0.0;
  }
  if (p.quiet_r[0] > 0) {
    const int all = __syncthreads_and(quiet);
    if (threadIdx.x == 0) cx.qpi[cx.tile] = all;
  }
}

// Stage 2, part 2 (tau_{n+1}): T^{n+1} = T^n + [(T' - T^n) + h R_T(e', u', pi^{n+1})]/2,
// root solve -> (e, u~)^{n+1} (written over e^n and u~^{n-1}), diagnostics.
// BK: P + Pi^{n+1} in T~ and in the root solve.  The root solve starts from e'
// in every guess mode (no network instance).
template <typename RT, int TX, int TY, int TZ, bool VISC, bool BK = false>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(s2t_waves<RT, TX, TY, TZ, BK>()))) void k_stage2_T(const EventDesc* __restrict__ evs,
                                                     GroupTable gt) {
  __shared__ RT lds[lds_doubles_allf<TX, TY, TZ>()];
  const Ctx cx = load_ctx(evs, gt, 1);
  const DFields& f = cx.f;
  const StepParams& p = cx.p;
  const EosDev& eos = cx.eos;
  const Geo& g = cx.g;
  const Pos q = cell_pos<TX, TY, TZ>(p, cx.tg, cx.tile);
  double v[kNP];
#pragma unroll
  for (int s = 0; s < kNP; ++s) v[s] = 0.0;
  const double tf = g.cart ? 1.0 : g.tau;
  if (tile_asleep<TX, TY, TZ>(p, cx.tg, cx.qcur, cx.tile)) {
    // the diagnostics the vacuum cells would give; T~ is unchanged
    v[P_CFL] = vacuum_cfl<RT>(p, tf) * p.h;
    if (q.active) {
      v[P_TSUM] = f.T[0][q.c];
      v[P_VAC] = 1.0;
      v[P_NEG] = f.T[0][q.c] < 0.0 ? 1.0 : 0.0;  // as the skipped root solve would count
    }
    block_partials(v, f.partial + (size_t)kNP * cx.tg.ntiles, cx.tg.ntiles, cx.tile);
    if (threadIdx.x == 0) cx.qnext[cx.tile] = 1;
    return;
  }
  constexpr int NT = BK ? 11 : 10;  // the components T~ uses: pi~ (and Pi)
  double R[BK ? 16 : 14];
  const double cfl = tile_divergence<RT, TX, TY, TZ, true, false, VISC ? 2 : 0, BK, false, true>(
      f.e1, f.u1, f.pi, p, eos, tf, q, R, lds);
  v[P_CFL] = cfl * p.h;
  double K[4] = {1.0, 0.0, 0.0, 0.0}, prev = 0.0, PiN = 0.0;
  const bool t1s = cx.t1same[cx.tile] != 0;
  if (q.active) {
    const int c = q.c;
    const double e1 = f.e1[c], u1 = f.u1[0][c], u2 = f.u1[1][c], u3 = f.u1[2][c];
    // where e' = 0 the regulator zeroed pi^{n+1} in stage 2pi (vac_zero): no loads
    double pc[NT];
#pragma unroll
    for (int m = 0; m < NT; ++m) pc[m] = 0.0;
    if (VISC && !(e1 == 0.0 && p.vac_zero)) {
#pragma unroll
      for (int m = 0; m < NT; ++m) pc[m] = ldq<RT>(f.pi[m], c);
    }
    if constexpr (BK) PiN = pc[10];
    if (!g.cart) {
      double P, cs2;
      eos_p_cs2(eos, e1, P, cs2);
      if constexpr (BK) P += PiN;
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
      // stage 1 left T~' = T~^n unstored in such a tile: the loaded value is
      // stale there and replaced (loading it anyway keeps the loads together)
      const double t1l = f.T1[nu][c];
      const double t1 = t1s ? t0 : t1l;
      Tn[nu] = t0 + 0.5 * ((t1 - t0) + p.h * R[nu]);
      // T~^{n+1} goes over T~^n: a value that is bitwise unchanged (a vacuum
      // tile's cells, where no flux or source acts) is already in memory
      if (__builtin_bit_cast(long long, Tn[nu]) != __builtin_bit_cast(long long, t0))
        st_cell(f.T[nu] + c, Tn[nu]);
    }
    const double inv_tf1 = 1.0 / (g.cart ? 1.0 : g.tau1);
#pragma unroll
    for (int nu = 0; nu < 4; ++nu) K[nu] = Tn[nu] * inv_tf1 - pc[nu];
    prev = e1;
    v[P_TSUM] = Tn[0];
  }
  // the predictor's e' starts the corrector's root solve whatever the guess mode:
  // the two stages' states differ by O(h^2), closer than the learned guess (on the
  // 64-event batch the network here cost 3% of the step and 0.004 iterations per
  // solve more than e')
  const double x0 = root_guess<false>(p, q.active, K[0], K[1], K[2], K[3], prev);
  bool quiet = true;  // this cell's part of the quiet-tile test
  if (q.active) {
    const int c = q.c;
    int it, fl;
    const Prim s = con2prim<BK>(eos, p, K[0], K[1], K[2], K[3], x0, it, fl, PiN);
    count_solve(v, it, fl);
    if (p.quiet_r[0] > 0)  // e before and after stage 1 (viscous: tested in stage2pi)
      quiet = VISC || (f.e[c] == 0.0 && prev == 0.0);
    quiet = quiet && s.e == 0.0 && !(K[0] >= p.eps_cut);
    st_cell(f.e + c, s.e);
    st_cell(f.up[0] + c, s.u1);  // becomes u~^{n+1} after the host swaps u and up
    st_cell(f.up[1] + c, s.u2);
    st_cell(f.up[2] + c, s.u3);
    v[P_EMAX] = s.e;
    v[P_VAC] = s.e == 0.0 ? 1.0 : 0.0;
  }
  if (p.quiet_r[0] > 0) {
    const int all = __syncthreads_and(quiet);
    if (threadIdx.x == 0) cx.qnext[cx.tile] = all && (!VISC || cx.qpi[cx.tile]);
  }
  block_partials(v, f.partial + (size_t)kNP * cx.tg.ntiles, cx.tg.ntiles, cx.tile);
}

// ---------------------------------------------------------------------------
// Tile shapes available to the launcher (the autotuner picks among them).
// ---------------------------------------------------------------------------
struct TileShape {
  int tx, ty, tz;
};
#define KTMI_TILE_LIST(X) \
  X(0, 4, 4, 16) X(1, 2, 8, 16) X(2, 4, 8, 8) X(3, 1, 8, 32) X(4, 16, 16, 1) X(5, 256, 1, 1)
#define KTMI_TILE_ENTRY(id, X, Y, Z) {X, Y, Z},
constexpr TileShape kTiles[] = {KTMI_TILE_LIST(KTMI_TILE_ENTRY)};
#undef KTMI_TILE_ENTRY
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

// Launchers of the stencil passes, one per (pass, arithmetic type), each
// defined in its own object (ktmi_stencil.hip built per pass and type).  `net`
// selects the instances whose root solves take the network's guess.  The
// passes that evaluate S_pi come twice: without and with the lambda_1 term
// (a compile-time choice, so the first-order kernels keep their registers), and
// the three viscous passes come once more with bulk pressure and baryon density.
enum Pass : int {
  PASS_FIRST = 0, PASS_STAGE1_V, PASS_STAGE1_I, PASS_STAGE2_PI, PASS_STAGE2_T_V, PASS_STAGE2_T_I,
  PASS_STAGE1_V_L1, PASS_STAGE2_PI_L1, PASS_STAGE1_BK, PASS_STAGE2_PI_BK, PASS_STAGE2_T_BK,
  PASS_COUNT
};
typedef void (*PassLauncher)(hipStream_t s, int tile, bool net, const EventDesc* evs,
                             const GroupTable& gt);
#define KTMI_DECLARE_PASS(P)                                                               \
  void launch_pass##P##_f64(hipStream_t, int, bool, const EventDesc*, const GroupTable&); \
  void launch_pass##P##_f32(hipStream_t, int, bool, const EventDesc*, const GroupTable&);
KTMI_DECLARE_PASS(0)
KTMI_DECLARE_PASS(1)
KTMI_DECLARE_PASS(2)
KTMI_DECLARE_PASS(3)
KTMI_DECLARE_PASS(4)
KTMI_DECLARE_PASS(5)
KTMI_DECLARE_PASS(6)
KTMI_DECLARE_PASS(7)
KTMI_DECLARE_PASS(8)
KTMI_DECLARE_PASS(9)
KTMI_DECLARE_PASS(10)
#undef KTMI_DECLARE_PASS

}  // namespace ktmi
