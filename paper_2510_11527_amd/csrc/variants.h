// variants.h -- stage-kernel tile variants per dimension (index 0 = default).
#pragma once
#include "launch.h"

namespace af4 {

// 1D: two cells per thread measured fastest (more work per barrier)
#define AF4_VARIANTS_D1(X) X(0, 512, 1, 1, 256, "generic-512") X(1, 256, 1, 1, 256, "generic-256") \
    X(2, 128, 1, 1, 128, "generic-128")
// 2D: KIND 4 = thread-owned-items kernel for fluxes c1 u + c2 u^2 and
// Buckley-Leverett fluxes (periodic or open ends), 1 = tuned kernel with a
// {u,a,f_x,f_y} half-grid table (any flux, periodic), 2 = tuned kernel with a
// {u,a} table (fluxes c1 u + c2 u^2, periodic), 0 = generic kernel (the only
// one with SI blending)
#define AF4_VARIANTS_D2(X)                                                                          \
    X(0, 32, 16, 1, 256, 4, "2d-own-32x16") X(1, 32, 8, 1, 128, 4, "2d-own-32x8")                    \
    X(2, 32, 16, 1, 256, 1, "2d-table4-32x16") X(3, 32, 8, 1, 128, 1, "2d-table4-32x8")              \
    X(4, 32, 16, 1, 256, 2, "2d-table2-32x16") X(5, 32, 8, 1, 256, 0, "generic-32x8")                \
    X(6, 16, 16, 1, 256, 0, "generic-16x16") X(7, 32, 32, 1, 512, 4, "2d-own-32x32")
// the tile variant whose generic kernel also has the limiter-counting form
// (af_limiter_activity)
constexpr int count_variant(int dim) { return dim == 2 ? 5 : dim == 3 ? 6 : 0; }

// 3D: KIND 1 = the kernel that marches along z (fluxes c1 u + c2 u^2; TZ is
// the number of cell planes a workgroup walks: longer walks re-read fewer
// planes below their first, shorter ones give small grids more workgroups;
// two threads per (x, y) column), 0 = generic kernel (any flux).  The
// generic 8x8x8 tile (125 KiB of LDS with SI blending in FP32) does not fit
// in FP64, where 8x8x4 is the first generic tile built.
#define AF4_VARIANTS_D3(X)                                                                            \
    X(0, 16, 8, 32, 256, 1, "3d-march-16x8x32") X(1, 16, 8, 64, 256, 1, "3d-march-16x8x64")            \
    X(2, 8, 8, 32, 128, 1, "3d-march-8x8x32") X(3, 16, 8, 128, 256, 1, "3d-march-16x8x128")            \
    X(4, 16, 8, 256, 256, 1, "3d-march-16x8x256") X(5, 8, 8, 8, 512, 0, "generic-8x8x8")                  \
    X(6, 8, 8, 4, 256, 0, "generic-8x8x4") X(7, 8, 4, 4, 128, 0, "generic-8x4x4")                       \
    X(8, 4, 4, 4, 64, 0, "generic-4x4x4")

}  // namespace af4
