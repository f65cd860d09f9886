// ktmi_spectra.hpp -- arguments and launcher of the smooth Cooper-Frye spectra
// kernels (ktmi_spectra.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "ktmi_device.hpp"
#include "ktmi_surface.hpp"

namespace ktmi {

constexpr int kMaxSlices = 64;  // element slices summed by the fold kernel

struct SpectraArgs {
  const double* elements;  // n surface records of kSurfRec doubles
  long n;
  double T, eps_plus_P;    // freeze-out temperature; e + P for delta f (0: none)
  int ns, nY, npt, nphi;
  long nbins;              // ns nY npt nphi
  const double* tables;    // mass, dof, stat, mu (ns each), Y, pT, cos phi, sin phi
  double* partial;         // spectra_slices(n) x nbins
  double* out;             // nbins
};

int spectra_slices(long n);
int launch_spectra(const SpectraArgs& a, hipStream_t s);

}  // namespace ktmi
