// FDK reconstruction of a compensated scan: per-view constants, the volume
// grid and the launcher (kernels in fdk.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ecc_internal.hpp"

namespace ecc {

// Per-view constants of the FDK reconstruction (FP32).
struct FdkView {
    float P[12];              // moved P' = P T(theta), rows 0-1 about the principal point
    float beta, delta;        // orbit angle from the first view; (scan range - pi) / 2
    float f, u0, v0;          // intrinsics (pixels)
    float scale, inv_tau;     // dbeta D^2; f / D (1 / pixel pitch at the isocentre)
    float pad;
};
static_assert(sizeof(FdkView) == 80, "FdkView layout");

// Reconstruction grid: nx x ny x nz voxels of voxel_mm centred on the isocentre.
struct FdkVolume {
    int32_t nx, ny, nz;
    float voxel_mm;
};

// pw: [n_views][W] scratch for the Parker weights; xw: [n_views H][W] scratch
// for the weighted rows (split by column parity); Qi: the filtered views.
hipError_t launch_fdk(const float *images, const ViewGeom *nominal, const ViewGeom *moved, int n_views, int W,
                      int H, FdkVolume vol, FdkView *views, float *pw, float *xw, float2 *Qi, float *out,
                      hipStream_t s);

}  // namespace ecc
