// ktmi_spectra.hip -- smooth Cooper-Frye spectra on the GPU (arXiv:1802.04449,
// Sec. IV, eq. cooper_frye with f_eq and delta f of eqn. feq; App. A.2: the sum
// over surface elements runs on the GPU, elements shared inside a workgroup).
//
// dN/(dY pT dpT dphi) = g / (2 pi hbarc)^3 sum_elements p^mu dSigma_mu f (1 + df)
// for every (species, Y, pT, phi) bin, with (tilde components, element centre
// (tau, eta_s)) p~ = (m_T cosh(Y - eta_s), pT cos phi, pT sin phi, m_T sinh(Y - eta_s)),
// p^mu dSigma_mu = p~^tau dS_tau + p~^x dS_x + p~^y dS_y + (p~^eta / tau) dS_eta,
// p.u = p~^tau u~^tau - p~^x u~^x - p~^y u~^y - p~^eta u~^eta,
// f = 1 / (exp((p.u - mu)/T) + sigma), df = (1 - sigma f) p~_a p~_b pi~^{ab} / (2 T^2 (e + P)).
//
// Layout of the work: a thread owns kPhi consecutive phi bins of one (species, Y,
// pT); a workgroup holds 256 such threads and one slice of the elements, which it
// streams through LDS in chunks (every element is read from memory once per
// workgroup and used by all its bins).  Slices give the chip enough workgroups;
// their partial sums are added in slice order by a second kernel, so the result
// does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <math.h>

#include <vector>

#include "../../include/ktmi.h"
#include "ktmi_spectra.hpp"

namespace ktmi {

namespace {

constexpr int kSpecBlock = 256;
#ifndef KTMI_SPEC_PHI
#define KTMI_SPEC_PHI 16
#endif
// phi bins per thread; on the 201x201x105 benchmark surface (41660 elements, 8
// species, 41 x 15 x 48 bins): 4 -> 30.0 ms, 8 -> 24.4 ms, 16 -> 23.7 ms
constexpr int kPhi = KTMI_SPEC_PHI;
constexpr int kChunk = 128; // elements per LDS chunk
constexpr int kElemVals = 20;

__global__ __launch_bounds__(kSpecBlock) void k_spectra(SpectraArgs a) {
  __shared__ double sel[kChunk][kElemVals];
  const gdouble* el = (const gdouble*)a.elements;
  const gdouble* tab = (const gdouble*)a.tables;
  const int nchunk_phi = (a.nphi + kPhi - 1) / kPhi;
  const long nthr = (long)a.ns * a.nY * a.npt * nchunk_phi;
  const long b = (long)blockIdx.x * kSpecBlock + threadIdx.x;
  const bool act = b < nthr;
  const long bb = act ? b : 0;
  const int ic = (int)(bb % nchunk_phi);
  const int ip = (int)((bb / nchunk_phi) % a.npt);
  const int iy = (int)((bb / ((long)nchunk_phi * a.npt)) % a.nY);
  const int s = (int)(bb / ((long)nchunk_phi * a.npt * a.nY));
  // tables: mass, dof, stat, mu (ns each), Y (nY), pT (npt), cos phi, sin phi (nphi each)
  const double m = tab[s], sig = tab[2 * a.ns + s], mu = tab[3 * a.ns + s];
  const double Y = tab[4 * a.ns + iy];
  const double pt = tab[4 * a.ns + a.nY + ip];
  const gdouble* cphi = tab + 4 * a.ns + a.nY + a.npt;
  const gdouble* sphi = cphi + a.nphi;
  const double mT = sqrt(m * m + pt * pt);
  double px[kPhi], py[kPhi], acc[kPhi];
#pragma unroll
  for (int q = 0; q < kPhi; ++q) {
    const int iq = ic * kPhi + q;
    const bool ok = iq < a.nphi;
    px[q] = ok ? pt * cphi[iq] : 0.0;
    py[q] = ok ? pt * sphi[iq] : 0.0;
    acc[q] = 0.0;
  }
  const double invT = 1.0 / a.T;
  const bool with_df = a.eps_plus_P > 0.0;
  const double dfc = with_df ? 1.0 / (2.0 * a.T * a.T * a.eps_plus_P) : 0.0;
  // this workgroup's slice of the elements
  const long per = (a.n + gridDim.y - 1) / gridDim.y;
  const long e0 = (long)blockIdx.y * per;
  const long e1 = e0 + per < a.n ? e0 + per : a.n;
  for (long c0 = e0; c0 < e1; c0 += kChunk) {
    const int cn = (int)(e1 - c0 < kChunk ? e1 - c0 : kChunk);
    __syncthreads();
    for (int k = threadIdx.x; k < cn * kElemVals; k += kSpecBlock) {
      const int e = k / kElemVals, v = k % kElemVals;
      // stored: tau, eta, dS (4), u~ (3), pi~ (10), spare
      const int src = v == 0 ? 1 : (v == 1 ? 4 : v + 3);
      sel[e][v] = v < 19 ? el[(c0 + e) * kSurfRec + src] : 0.0;
    }
    __syncthreads();
    if (!act) continue;
    for (int e = 0; e < cn; ++e) {
      const double tau = sel[e][0], eta = sel[e][1];
      const double dS0 = sel[e][2], dS1 = sel[e][3], dS2 = sel[e][4], dS3 = sel[e][5];
      const double ux = sel[e][6], uy = sel[e][7], ue = sel[e][8];
      const double ut = sqrt(1.0 + ux * ux + uy * uy + ue * ue);
      const double yrel = Y - eta;
      const double p0 = mT * cosh(yrel), p3 = mT * sinh(yrel);
      const double pdS_l = p0 * dS0 + p3 / tau * dS3;  // longitudinal part of p.dSigma
      const double pu_l = p0 * ut - p3 * ue;
      double pi00 = 0, pi01 = 0, pi02 = 0, pi03 = 0, pi11 = 0, pi12 = 0, pi13 = 0, pi22 = 0,
             pi23 = 0, pi33 = 0;
      if (with_df) {
        pi00 = sel[e][9];
        pi01 = sel[e][10];
        pi02 = sel[e][11];
        pi03 = sel[e][12];
        pi11 = sel[e][13];
        pi12 = sel[e][14];
        pi13 = sel[e][15];
        pi22 = sel[e][16];
        pi23 = sel[e][17];
        pi33 = sel[e][18];
      }
#pragma unroll
      for (int q = 0; q < kPhi; ++q) {
        const double pdS = pdS_l + px[q] * dS1 + py[q] * dS2;
        const double pu = pu_l - px[q] * ux - py[q] * uy;
        const double f = 1.0 / (exp((pu - mu) * invT) + sig);
        double w = 1.0;
        if (with_df) {
          // p~_a p~_b pi~^{ab} with p~_a = (p0, -px, -py, -p3)
          const double x = px[q], y = py[q];
          const double ppi = p0 * p0 * pi00 + x * x * pi11 + y * y * pi22 + p3 * p3 * pi33 +
                             2.0 * (-p0 * x * pi01 - p0 * y * pi02 - p0 * p3 * pi03 + x * y * pi12 +
                                    x * p3 * pi13 + y * p3 * pi23);
          w = 1.0 + (1.0 - sig * f) * ppi * dfc;
        }
        acc[q] += pdS * f * w;
      }
    }
  }
  if (!act) return;
  gdouble* part = (gdouble*)a.partial + (long)blockIdx.y * a.nbins;
#pragma unroll
  for (int q = 0; q < kPhi; ++q) {
    const int iq = ic * kPhi + q;
    if (iq < a.nphi) part[(((long)s * a.nY + iy) * a.npt + ip) * a.nphi + iq] = acc[q];
  }
}

// out[bin] = dof[s] / (2 pi hbarc)^3 * sum over slices (in slice order).
__global__ __launch_bounds__(kSpecBlock) void k_spectra_fold(SpectraArgs a, int nslice) {
  const long bin = (long)blockIdx.x * kSpecBlock + threadIdx.x;
  if (bin >= a.nbins) return;
  const gdouble* part = (const gdouble*)a.partial;
  const gdouble* tab = (const gdouble*)a.tables;
  double sum = 0.0;
  for (int k = 0; k < nslice; ++k) sum += part[(long)k * a.nbins + bin];
  const int s = (int)(bin / ((long)a.nY * a.npt * a.nphi));
  const double pref = 1.0 / ((2.0 * M_PI * kHbarc) * (2.0 * M_PI * kHbarc) * (2.0 * M_PI * kHbarc));
  ((gdouble*)a.out)[bin] = tab[a.ns + s] * pref * sum;
}

}  // namespace

int spectra_slices(long n) {
  const long s = (n + 2 * kChunk - 1) / (2 * kChunk);  // at least two chunks per slice
  return (int)(s < 1 ? 1 : (s > kMaxSlices ? kMaxSlices : s));
}

int launch_spectra(const SpectraArgs& a, hipStream_t s) {
  const int nslice = spectra_slices(a.n);
  const long nthr = (long)a.ns * a.nY * a.npt * ((a.nphi + kPhi - 1) / kPhi);
  const long gx = (nthr + kSpecBlock - 1) / kSpecBlock;
  hipLaunchKernelGGL(k_spectra, dim3((unsigned)gx, (unsigned)nslice), dim3(kSpecBlock), 0, s, a);
  const long fx = (a.nbins + kSpecBlock - 1) / kSpecBlock;
  hipLaunchKernelGGL(k_spectra_fold, dim3((unsigned)fx), dim3(kSpecBlock), 0, s, a, nslice);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace ktmi

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
using namespace ktmi;

static size_t spectra_table_doubles(int ns, int nY, int npt, int nphi) {
  return ((size_t)4 * ns + nY + npt + 2 * (size_t)nphi + 31) / 32 * 32;
}

extern "C" {

size_t ktmi_spectra_workspace_bytes(long n, int ns, int nY, int npt, int nphi) {
  if (n < 0 || ns < 1 || nY < 1 || npt < 1 || nphi < 1) return 0;
  const size_t nbins = (size_t)ns * nY * npt * nphi;
  return (spectra_table_doubles(ns, nY, npt, nphi) + (size_t)spectra_slices(n) * nbins) *
         sizeof(double);
}

int ktmi_spectra(const double* elements, long n, double T, double eps_plus_P, int ns,
                 const double* mass, const double* dof, const int* stat, const double* mu, int nY,
                 const double* Y, int npt, const double* pt, int nphi, const double* phi,
                 double* out, void* ws, size_t ws_bytes, void* stream) {
  if (n < 0 || (n > 0 && !elements) || !(T > 0) || !(eps_plus_P >= 0) || ns < 1 || nY < 1 ||
      npt < 1 || nphi < 1 || !mass || !dof || !stat || !mu || !Y || !pt || !phi || !out || !ws)
    return KTMI_EINVAL;
  if (ws_bytes < ktmi_spectra_workspace_bytes(n, ns, nY, npt, nphi)) return KTMI_EINVAL;
  for (int s = 0; s < ns; ++s)
    if (!(mass[s] >= 0) || stat[s] < -1 || stat[s] > 1) return KTMI_EINVAL;
  std::vector<double> tab(spectra_table_doubles(ns, nY, npt, nphi), 0.0);
  for (int s = 0; s < ns; ++s) {
    tab[s] = mass[s];
    tab[ns + s] = dof[s];
    tab[2 * ns + s] = (double)stat[s];
    tab[3 * ns + s] = mu[s];
  }
  for (int i = 0; i < nY; ++i) tab[4 * ns + i] = Y[i];
  for (int i = 0; i < npt; ++i) tab[4 * ns + nY + i] = pt[i];
  for (int i = 0; i < nphi; ++i) {
    tab[4 * ns + nY + npt + i] = cos(phi[i]);
    tab[4 * ns + nY + npt + nphi + i] = sin(phi[i]);
  }
  hipStream_t st = (hipStream_t)stream;
  double* dtab = (double*)ws;
  if (hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, st) !=
      hipSuccess)
    return KTMI_EHIP;
  // the host table must outlive the copy
  if (hipStreamSynchronize(st) != hipSuccess) return KTMI_EHIP;
  SpectraArgs a;
  a.elements = elements;
  a.n = n;
  a.T = T;
  a.eps_plus_P = eps_plus_P;
  a.ns = ns;
  a.nY = nY;
  a.npt = npt;
  a.nphi = nphi;
  a.nbins = (long)ns * nY * npt * nphi;
  a.tables = dtab;
  a.partial = dtab + tab.size();
  a.out = out;
  return launch_spectra(a, st) == 0 ? KTMI_OK : KTMI_EHIP;
}

}  // extern "C"
