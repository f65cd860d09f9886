// ktmi_surface.hip -- freeze-out hypersurface finder on the GPU (arXiv:1802.04449,
// Sec. IV: surface elements dSigma_mu of constant freeze-out energy density e_f;
// App. A.2: the surface is found on the device between stored time slices, so
// the fields never travel to the host).
//
// One thread per hypercube of 2 x 2 x 2 x 2 grid points (two slices, two
// neighbouring cells per axis; an axis with one cell spans that cell's width).
// With phi = e - e_f at its 16 corners, the surface inside the hypercube is the
// zero set of the piecewise-linear interpolant of phi on the Kuhn triangulation.
// By the divergence theorem over the hot part (phi > 0) of the hypercube, the
// surface covector pointing out of the hot region is
//   S_mu = V_mu (f_lo(mu) - f_hi(mu)),
// V_mu the coordinate volume of the 3-faces normal to axis mu and f the hot
// volume fraction of a face: the mean over its six Kuhn tetrahedra of the exact
// fraction of a linear function.  Neighbouring hypercubes share faces, so sums
// of S telescope exactly.  dSigma_mu = tau_c S_mu (1 in Cartesian mode), tau_c
// the time of the element's centre: the mean of the sign changes along the 32
// edges; e, u~ and pi~ there are multilinear interpolants of the corners.
//
// Passes: a light count (one thread per hypercube, e only) of the hypercubes
// that straddle e_f per workgroup, an exclusive prefix sum of those counts, a
// compaction that writes each straddling hypercube's index to its slot, and the
// element pass over the slots, densely packed, so the heavy arithmetic runs only
// where there is surface.  No atomics: records come out in hypercube order, and
// the arithmetic is written in a fixed order with contraction off, so the output
// is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ktmi_surface.hpp"

#pragma clang fp contract(off)

namespace ktmi {

namespace {

constexpr int kSurfBlock = 256;

// Hot fraction of a tetrahedron on which phi is linear (vertex values v0..v3).
// The hot and cold vertices are taken in vertex order; every branch is a sum or
// product of positive terms.
__device__ __forceinline__ double tet_hot(double v0, double v1, double v2, double v3) {
  const double v[4] = {v0, v1, v2, v3};
  double p0 = 0.0, p1 = 0.0, p2 = 0.0, n0 = 0.0, n1 = 0.0, n2 = 0.0;
  int np = 0, nn = 0;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const bool hot = v[t] > 0.0;
    const double x = hot ? v[t] : -v[t];
    if (hot) {
      p0 = np == 0 ? x : p0;
      p1 = np == 1 ? x : p1;
      p2 = np == 2 ? x : p2;
      ++np;
    } else {
      n0 = nn == 0 ? x : n0;
      n1 = nn == 1 ? x : n1;
      n2 = nn == 2 ? x : n2;
      ++nn;
    }
  }
  if (np == 0) return 0.0;
  if (np == 4) return 1.0;
  if (np == 1) {
    const double a = p0;
    return (a / (a + n0)) * (a / (a + n1)) * (a / (a + n2));
  }
  if (np == 3) {
    const double c = n0;
    if (c == 0.0) return 1.0;
    return 1.0 - (c / (p0 + c)) * (c / (p1 + c)) * (c / (p2 + c));
  }
  // two hot (a, b) and two cold (c, d, magnitudes): the volume of {phi > 0} is
  // [a^2 b^2 + a b (a + b)(c + d) + c d (a^2 + a b + b^2)] / [(a+c)(a+d)(b+c)(b+d)]
  const double a = p0, b = p1, c = n0, d = n1;
  const double num = a * a * b * b + a * b * (a + b) * (c + d) + c * d * (a * a + a * b + b * b);
  const double den = (a + c) * (a + d) * (b + c) * (b + d);
  return num / den;
}

// Hot fraction of a 3-cube with corner values w[4 b0 + 2 b1 + b2]: mean over the
// Kuhn tetrahedra 000 -> +e_p -> +e_q -> 111 for the axis orders
// (0,1,2), (0,2,1), (1,0,2), (1,2,0), (2,0,1), (2,1,0).
__device__ __forceinline__ double cube_hot(const double w[8]) {
  double s = 0.0;
  s += tet_hot(w[0], w[4], w[6], w[7]);  // 0,1,2
  s += tet_hot(w[0], w[4], w[5], w[7]);  // 0,2,1
  s += tet_hot(w[0], w[2], w[6], w[7]);  // 1,0,2
  s += tet_hot(w[0], w[2], w[3], w[7]);  // 1,2,0
  s += tet_hot(w[0], w[1], w[5], w[7]);  // 2,0,1
  s += tet_hot(w[0], w[1], w[3], w[7]);  // 2,1,0
  return s / 6.0;
}

// Corner index of the hypercube (8 b_tau + 4 b_x + 2 b_y + b_eta) of bit b of
// the face normal to axis mu on side `side` (the face's bits run over the other
// three axes in increasing order).
__host__ __device__ constexpr int face_corner(int mu, int side, int b) {
  int c = 0, t = 0;
  for (int ax = 0; ax < 4; ++ax) {
    int bit = 0;
    if (ax == mu) {
      bit = side;
    } else {
      bit = (b >> (2 - t)) & 1;
      ++t;
    }
    c |= bit << (3 - ax);
  }
  return c;
}

// Hypercube index -> (i, j, k) and the flat cell index of its 8 spatial corners
// (grids hold fewer than 2^31 cells).
struct Cube {
  int i, j, k;
  int cell[8];
};

__device__ __forceinline__ Cube cube_of(const SurfaceArgs& a, int id) {
  const int cy = a.ny > 1 ? a.ny - 1 : 1, cz = a.ne > 1 ? a.ne - 1 : 1;
  Cube q;
  const int r = id / cz;
  q.k = id - r * cz;
  q.i = r / cy;
  q.j = r - q.i * cy;
  const int ii[2] = {q.i, a.nx > 1 ? q.i + 1 : q.i};
  const int jj[2] = {q.j, a.ny > 1 ? q.j + 1 : q.j};
  const int kk[2] = {q.k, a.ne > 1 ? q.k + 1 : q.k};
#pragma unroll
  for (int b = 0; b < 8; ++b) q.cell[b] = (ii[(b >> 2) & 1] * a.ny + jj[(b >> 1) & 1]) * a.ne + kk[b & 1];
  return q;
}

__host__ __device__ __forceinline__ long cube_count(long nx, long ny, long ne) {
  return (nx > 1 ? nx - 1 : 1) * (ny > 1 ? ny - 1 : 1) * (ne > 1 ? ne - 1 : 1);
}

// Whether hypercube id's 16 corners straddle e_f (some > e_f, some not).
__device__ __forceinline__ bool straddles(const SurfaceArgs& a, int id) {
  const gdouble* A = (const gdouble*)a.A;
  const gdouble* B = (const gdouble*)a.B;
  const Cube q = cube_of(a, id);
  int nhot = 0;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const gdouble* S = (c & 8) ? B : A;
    nhot += (S[q.cell[c & 7]] - a.eps_f) > 0.0;
  }
  return nhot != 0 && nhot != 16;
}

// Every count / compaction workgroup covers kSpan consecutive hypercubes: kIt
// rounds of kSurfBlock threads.  Scratch layout (words): [0, nblk) counts per
// workgroup, then exclusive offsets in place; [nblk, nblk + kIt kWaves nblk) the
// straddle mask of every (workgroup, round, wave).
constexpr int kWaves = kSurfBlock / 64;
constexpr int kIt = 16;
constexpr long kSpan = (long)kIt * kSurfBlock;

// Workgroup b of a launch of G runs on XCD b % 8; the span it takes is
// xcd_span(b, G): the spans [k G/8, (k+1) G/8) (remainder spread over the first
// XCDs) go to XCD k in order, so the planes a workgroup shares with the next
// span stay in one XCD's L2.  A bijection on [0, G).
__device__ __forceinline__ long xcd_span(long b, long G) {
  const long per = G / 8, rem = G % 8, k = b % 8;
  return k * per + (k < rem ? k : rem) + b / 8;
}

// Pass 1: straddle masks and straddling hypercubes per workgroup.
__global__ __launch_bounds__(kSurfBlock) void k_surface_count(SurfaceArgs a, int nblk) {
  __shared__ int wc[kWaves];
  const long ncube = cube_count(a.nx, a.ny, a.ne);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  gullong* blk = (gullong*)a.blocks;
  const long sb = xcd_span(blockIdx.x, nblk);
  gullong* masks = blk + nblk + sb * kIt * kWaves;
  int nw = 0;
  for (int it = 0; it < kIt; ++it) {
    const long id = sb * kSpan + (long)it * kSurfBlock + threadIdx.x;
    const bool cross = id < ncube && straddles(a, (int)id);
    const unsigned long long mask = __ballot(cross);
    if (lane == 0) masks[it * kWaves + wave] = mask;
    nw += __popcll(mask);
  }
  if (lane == 0) wc[wave] = nw;
  __syncthreads();
  if (threadIdx.x == 0) {
    int n = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) n += wc[w];
    blk[sb] = (unsigned long long)n;
  }
}

// Pass 2 (one workgroup of 1024): exclusive prefix sums of the counts, in place
// (each thread sums a run of consecutive counts, one workgroup-wide scan of the
// run totals, then each thread writes its run), and the total into *count.
__global__ __launch_bounds__(1024) void k_surface_offsets(SurfaceArgs a, int nblk) {
  __shared__ long long part[16];
  gullong* blk = (gullong*)a.blocks;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (nblk + 1023) / 1024;
  const int i0 = tid * per;
  long long loc = 0;
  for (int q = 0; q < per; ++q)
    if (i0 + q < nblk) loc += (long long)blk[i0 + q];
  long long x = loc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) part[wave] = x;
  __syncthreads();
  if (wave == 0) {
    long long p = lane < 16 ? part[lane] : 0;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const long long y = __shfl_up(p, o);
      if (lane >= o) p += y;
    }
    if (lane < 16) part[lane] = p;
  }
  __syncthreads();
  long long run = x - loc + (wave ? part[wave - 1] : 0);  // exclusive
  for (int q = 0; q < per; ++q)
    if (i0 + q < nblk) {
      const long long v = (long long)blk[i0 + q];
      blk[i0 + q] = (unsigned long long)run;
      run += v;
    }
  if (tid == 1023) *(gullong*)a.count = (unsigned long long)run;
}

// Pass 3: every straddling hypercube writes its index to its slot, in hypercube
// order (workgroup offset, then round, wave and lane), from the pass-1 masks.
__global__ __launch_bounds__(kSurfBlock) void k_surface_compact(SurfaceArgs a, int nblk) {
  __shared__ long long moff[kIt * kWaves];
  const gullong* blk = (const gullong*)a.blocks;
  const long sb = xcd_span(blockIdx.x, nblk);
  const gullong* masks = blk + nblk + sb * kIt * kWaves;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (wave == 0) {  // exclusive offsets of the kIt * kWaves masks (one wave, 64 masks)
    static_assert(kIt * kWaves == 64, "one mask per lane");
    const long long c = __popcll(masks[lane]);
    long long x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const long long y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    moff[lane] = (long long)blk[sb] + x - c;
  }
  __syncthreads();
  for (int it = 0; it < kIt; ++it) {
    const unsigned long long mask = masks[it * kWaves + wave];
    if (!((mask >> lane) & 1ull)) continue;
    const long long slot = moff[it * kWaves + wave] + __popcll(mask & ((1ull << lane) - 1ull));
    const long id = sb * kSpan + (long)it * kSurfBlock + threadIdx.x;
    if (slot < (long long)a.capacity) ((gdouble*)a.out)[slot * kSurfRec] = (double)id;
  }
}

// Pass 4: the element of every claimed slot below min(count, capacity).  Eight
// lanes share one element: the 16 corner values go through LDS, lane t
// evaluates the hot fraction of the 3-face normal to axis t/2 on side t%2 (its
// six tetrahedra) and the even lane of each pair forms S_mu; every lane forms the
// centre and the corner weights (the same arithmetic in each); lane t
// interpolates fields t and t + 8.  Grid-stride over groups of elements; the
// loop bound is block-uniform, so every thread reaches each barrier.
constexpr int kGroup = 8;
constexpr int kElemPerBlock = kSurfBlock / kGroup;

__global__ __launch_bounds__(kSurfBlock) void k_surface_elem(SurfaceArgs a) {
  __shared__ double sphi[kElemPerBlock][16];
  const gdouble* A = (const gdouble*)a.A;
  const gdouble* B = (const gdouble*)a.B;
  gdouble* outp = (gdouble*)a.out;
  const unsigned long long found = *(const gullong*)a.count;
  const long n = (long)(found < (unsigned long long)a.capacity ? found
                                                                : (unsigned long long)a.capacity);
  const int t = threadIdx.x & (kGroup - 1), g = threadIdx.x / kGroup;
  const int mu = t >> 1, side = t & 1;
  const double ext[4] = {a.tauB - a.tauA, a.dx, a.dy, a.de};
  const long ncell = (long)a.nx * a.ny * a.ne;
  // contiguous runs of element groups per workgroup, the runs of one XCD adjacent
  // (neighbouring elements share corner cells); the first min(grid, groups)
  // workgroups share the groups, so every XCD gets work
  const long ngrp = (n + kElemPerBlock - 1) / kElemPerBlock;
  const long G = (long)gridDim.x < ngrp ? (long)gridDim.x : ngrp;
  if ((long)blockIdx.x >= G) return;  // whole workgroup: before any barrier
  const long per = (ngrp + G - 1) / G, g0 = xcd_span(blockIdx.x, G) * per;
  const long g1 = g0 + per < ngrp ? g0 + per : ngrp;
  for (long base = g0 * kElemPerBlock; base < g1 * kElemPerBlock; base += kElemPerBlock) {
    const long slot = base + g;
    const bool act = slot < n;
    gdouble* r = outp + (act ? slot : 0) * kSurfRec;
    const int id = act ? (int)r[0] : 0;
    const Cube q = cube_of(a, id);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int c = 2 * t + u;
      const gdouble* S = (c & 8) ? B : A;
      sphi[g][c] = S[q.cell[c & 7]] - a.eps_f;
    }
    __syncthreads();
    double w[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) w[b] = sphi[g][face_corner(mu, side, b)];
    const double f = cube_hot(w);
    const double f_other = __shfl_xor(f, 1);
    double phi[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) phi[c] = sphi[g][c];
    double cen[4] = {0.0, 0.0, 0.0, 0.0};
    int ncross = 0;
#pragma unroll
    for (int c = 0; c < 16; ++c)
#pragma unroll
      for (int ax = 0; ax < 4; ++ax) {
        const int bitm = 1 << (3 - ax);
        if (c & bitm) continue;
        const int c2 = c | bitm;
        if ((phi[c] > 0.0) == (phi[c2] > 0.0)) continue;
        const double s = phi[c] / (phi[c] - phi[c2]);
#pragma unroll
        for (int a2 = 0; a2 < 4; ++a2) {
          const int bb = (c >> (3 - a2)) & 1;
          cen[a2] += (a2 == ax) ? s : (double)bb;
        }
        ++ncross;
      }
#pragma unroll
    for (int a2 = 0; a2 < 4; ++a2) cen[a2] /= (double)ncross;
    const double tc = a.tauA + cen[0] * ext[0];
    if (act) {
      if (side == 0) {  // S_mu = V_mu (f_lo - f_hi), V_mu over the other axes in order
        double V = 1.0;
#pragma unroll
        for (int ax = 0; ax < 4; ++ax)
          if (ax != mu) V *= ext[ax];
        r[5 + mu] = (a.cart ? 1.0 : tc) * (V * (f - f_other));
      }
      if (t == 0) {
        r[1] = tc;
        r[2] = ((double)q.i - 0.5 * (a.nx - 1)) * a.dx + (a.nx > 1 ? cen[1] * a.dx : 0.0);
        r[3] = ((double)q.j - 0.5 * (a.ny - 1)) * a.dy + (a.ny > 1 ? cen[2] * a.dy : 0.0);
        r[4] = ((double)q.k - 0.5 * (a.ne - 1)) * a.de + (a.ne > 1 ? cen[3] * a.de : 0.0);
        r[23] = 0.0;
      }
      double wgt[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        double wv = 1.0;
#pragma unroll
        for (int a2 = 0; a2 < 4; ++a2) {
          const int bb = (c >> (3 - a2)) & 1;
          wv *= bb ? cen[a2] : 1.0 - cen[a2];
        }
        wgt[c] = wv;
      }
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
        const int fld = t + kGroup * h2;
        if (fld >= 14) continue;
        double v = 0.0;
        if (fld < a.nf) {
#pragma unroll
          for (int c = 0; c < 16; ++c) {
            const gdouble* S = (c & 8) ? B : A;
            v += wgt[c] * S[(long)fld * ncell + (long)q.cell[c & 7]];
          }
        }
        if (fld == 0)
          r[22] = v;
        else
          r[8 + fld] = v;  // u~ at 9..11, pi~ at 12..21
      }
    }
    __syncthreads();
  }
}

}  // namespace

size_t surface_scratch_words(long nx, long ny, long ne) {
  return (size_t)((cube_count(nx, ny, ne) + kSpan - 1) / kSpan) * (1 + kIt * kWaves) + 1;
}

int launch_surface(const SurfaceArgs& a, hipStream_t s) {
  const long nblk = (cube_count(a.nx, a.ny, a.ne) + kSpan - 1) / kSpan;
  hipLaunchKernelGGL(k_surface_count, dim3((unsigned)nblk), dim3(kSurfBlock), 0, s, a, (int)nblk);
  hipLaunchKernelGGL(k_surface_offsets, dim3(1), dim3(1024), 0, s, a, (int)nblk);
  if (a.capacity > 0) {
    hipLaunchKernelGGL(k_surface_compact, dim3((unsigned)nblk), dim3(kSurfBlock), 0, s, a,
                       (int)nblk);
    // enough workgroups for the buffer, at most 16 per CU's worth of the chip
    const long eb = std::min<long>((a.capacity + kElemPerBlock - 1) / kElemPerBlock, 4096);
    hipLaunchKernelGGL(k_surface_elem, dim3((unsigned)eb), dim3(kSurfBlock), 0, s, a);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ktmi
