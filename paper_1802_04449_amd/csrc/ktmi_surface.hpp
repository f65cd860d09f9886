// ktmi_surface.hpp -- arguments and launcher of the freeze-out hypersurface
// finder (ktmi_surface.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "ktmi_device.hpp"

namespace ktmi {

constexpr int kSurfRec = 24;  // doubles per surface element record

struct SurfaceArgs {
  int nx, ny, ne;
  double dx, dy, de;
  const double* A;  // slice at tauA: nf fields of nx*ny*ne (e, u~x, u~y, u~eta[, pi~ x10])
  const double* B;  // slice at tauB > tauA, same layout
  double tauA, tauB;
  int nf;           // 4 or 14
  double eps_f;
  int cart;         // 1: sqrt(-g) = 1
  double* out;      // capacity records of kSurfRec doubles
  long capacity;
  unsigned long long* count;   // number of elements found (may exceed capacity)
  unsigned long long* blocks;  // scratch: surface_scratch_words(nx, ny, ne) words
};

// Scratch words the finder needs for a grid (per-workgroup counts and offsets).
size_t surface_scratch_words(long nx, long ny, long ne);

// Launches the finder on stream s (count, then offsets, then the records); 0 on success.
int launch_surface(const SurfaceArgs& a, hipStream_t s);

}  // namespace ktmi
