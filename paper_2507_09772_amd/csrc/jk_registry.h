// jk_registry.h -- per-class launchers filled in by the kern_bra units.
#pragma once
#include <hip/hip_runtime.h>

#include "jk_device.h"

namespace jk {

constexpr int LMAX_BUILT = 3;  // classes instantiated up to (ff|ff)

using Launcher = hipError_t (*)(const JkArgs &, hipStream_t);

struct ClassEntry {
    Launcher tiles[2][2];  // [family - 1][0: FP64, 1: FP32], quartets from tiles
    Launcher list64[2];    // [family - 1], FP64 pass over the appended list
    Launcher ex64, ex32;   // export (default family)
};

// Indexed by class_id(li, lj, lk, ll); zero-initialised, filled by the
// static initialisers of the kernel units when the library loads.
extern ClassEntry g_classes[NCLS];

}  // namespace jk
