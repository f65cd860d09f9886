// ktmi_stencil.hip -- instances of one stencil pass of the RK2 step for one
// arithmetic type, and the launcher the host code calls for them.  The build
// compiles this file once per (pass, type) with -DKTMI_PASS=<0..10>
// -DKTMI_RT=<double|float> -DKTMI_LAUNCH_FN=launch_pass<P>_<f64|f32>, so the
// instances compile in parallel.  Passes: 0 first-step estimate, 1 / 2 stage 1
// (viscous / ideal), 3 stage 2 pi, 4 / 5 stage 2 T (viscous / ideal), 6 / 7
// stage 1 viscous / stage 2 pi with the second-order lambda_1 term, 8 / 9 / 10
// stage 1 / stage 2 pi / stage 2 T with bulk pressure and baryon density.
#include "ktmi_kernels.hpp"

#if !defined(KTMI_PASS) || !defined(KTMI_RT) || !defined(KTMI_LAUNCH_FN)
#error "build with -DKTMI_PASS, -DKTMI_RT and -DKTMI_LAUNCH_FN"
#endif

namespace ktmi {
namespace {

template <int X, int Y, int Z, bool N>
void launch_tile(dim3 g, dim3 b, hipStream_t s, const EventDesc* evs, const GroupTable& gt) {
#if KTMI_PASS == 0
  hipLaunchKernelGGL((k_first_estimate<KTMI_RT, X, Y, Z>), g, b, 0, s, evs, gt);
#elif KTMI_PASS == 1
  hipLaunchKernelGGL((k_stage1<KTMI_RT, X, Y, Z, true, N, false>), g, b, 0, s, evs, gt);
#elif KTMI_PASS == 2
  hipLaunchKernelGGL((k_stage1<KTMI_RT, X, Y, Z, false, N, false>), g, b, 0, s, evs, gt);
#elif KTMI_PASS == 3
  hipLaunchKernelGGL((k_stage2_pi<KTMI_RT, X, Y, Z, false>), g, b, 0, s, evs, gt);
#elif KTMI_PASS == 4
  hipLaunchKernelGGL((k_stage2_T<KTMI_RT, X, Y, Z, true>), g, b, 0, s, evs, gt);
#elif KTMI_PASS == 5
  hipLaunchKernelGGL((k_stage2_T<KTMI_RT, X, Y, Z, false>), g, b, 0, s, evs, gt);
#elif KTMI_PASS == 6
  hipLaunchKernelGGL((k_stage1<KTMI_RT, X, Y, Z, true, N, true>), g, b, 0, s, evs, gt);
#elif KTMI_PASS == 7
  hipLaunchKernelGGL((k_stage2_pi<KTMI_RT, X, Y, Z, true>), g, b, 0, s, evs, gt);
#elif KTMI_PASS == 8
  hipLaunchKernelGGL((k_stage1<KTMI_RT, X, Y, Z, true, false, false, true>), g, b, 0, s, evs, gt);
#elif KTMI_PASS == 9
  hipLaunchKernelGGL((k_stage2_pi<KTMI_RT, X, Y, Z, false, true>), g, b, 0, s, evs, gt);
#elif KTMI_PASS == 10
  hipLaunchKernelGGL((k_stage2_T<KTMI_RT, X, Y, Z, true, true>), g, b, 0, s, evs, gt);
#else
#error "KTMI_PASS out of range"
#endif
}

// only the stage-1 passes without bulk take the network's guess (stage 2T starts
// its root solve from the predictor's e; the other passes have no root solve)
constexpr bool kHasNet = KTMI_PASS == 1 || KTMI_PASS == 2 || KTMI_PASS == 6;

}  // namespace

// One launch over the tiles of every event in gt (events of one class).
void KTMI_LAUNCH_FN(hipStream_t s, int tile, bool net, const EventDesc* evs,
                    const GroupTable& gt) {
  const dim3 grid(gt.start[gt.nev]), block(kBlock);
  switch (tile) {
#define KTMI_TILE_CASE(id, X, Y, Z)                        \
  case id:                                                 \
    if (kHasNet && net)                                    \
      launch_tile<X, Y, Z, kHasNet>(grid, block, s, evs, gt); \
    else                                                   \
      launch_tile<X, Y, Z, false>(grid, block, s, evs, gt); \
    break;
    KTMI_TILE_LIST(KTMI_TILE_CASE)
#undef KTMI_TILE_CASE
    default:
      break;
  }
}

}  // namespace ktmi
