// variants.h -- stage-kernel tile variants per dimension (index 0 = default).
#pragma once
#include "launch.h"

namespace af4 {

#define AF4_VARIANTS_D1(X) X(0, 256, 1, 1, 256, "256") X(1, 128, 1, 1, 128, "128")
#define AF4_VARIANTS_D2(X) \
    X(0, 32, 8, 1, 256, "32x8") X(1, 16, 16, 1, 256, "16x16") X(2, 64, 4, 1, 256, "64x4") X(3, 32, 16, 1, 256, "32x16")
#define AF4_VARIANTS_D3(X) X(0, 8, 8, 4, 256, "8x8x4") X(1, 8, 4, 4, 128, "8x4x4") X(2, 4, 4, 4, 64, "4x4x4")

}  // namespace af4
