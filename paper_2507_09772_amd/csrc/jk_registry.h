// jk_registry.h -- per-class launchers filled in by the kern_bra units.
#pragma once
#include <hip/hip_runtime.h>

#include "jk_device.h"

namespace jk {

constexpr int LMAX_BUILT = 4;  // classes instantiated up to (gg|gg)

using Launcher = hipError_t (*)(const JkArgs &, hipStream_t);
// Batched builds: the tiles of many descriptors (molecules) in one launch.
using BatchLauncher = hipError_t (*)(const BatchDesc *, int ndesc, int total_tiles, hipStream_t);
using BatchRowLauncher = hipError_t (*)(const BatchDesc *, int ndesc, int total_tasks, size_t lds, hipStream_t);

struct ClassEntry {
    Launcher tiles[3][2];  // [family - 1][0: FP64, 1: FP32], quartets from tiles (none for family 3)
    Launcher ex64, ex32;   // export (default family)
    Launcher row[3][2];    // row mode, 256-lane workgroups (long bras), [family - 1][0: FP64, 1: FP32]
    Launcher srow[3][2];   // row mode, 64-lane workgroups (short bras)
    size_t row_fixed[3][2];  // row-mode LDS bytes per wave besides the K rows, [family - 1][precision]
    BatchLauncher batch[3][2];       // [family - 1][precision]
    BatchRowLauncher batch_row[3][2];  // 64-lane row tasks of many descriptors
};

// LDS bytes of one row-mode workgroup of nw waves: the fixed part (per wave;
// family 1 instead keeps the bra's npb primitive pair records) plus nset
// copies of the bra's K rows over ncols compressed columns and its J_IJ block.
inline size_t row_lds_bytes(const ClassEntry &e, int fam, int pr, int li, int lj, int nset, int ncols, int nw,
                            int npb) {
    return (size_t)nw * e.row_fixed[fam - 1][pr] + (fam == 1 ? sizeof(PrimPair) * (size_t)npb : 0) +
           sizeof(double) * (size_t)nset * ((size_t)(ncart(li) + ncart(lj)) * ncols + (size_t)ncart(li) * ncart(lj));
}

// LDS budget of one row-mode workgroup (dynamic shared memory; gfx950 has
// 160 KB per CU, kernels above 64 KB opt in through a function attribute).
constexpr int ROW_LDS_MAX = 128 * 1024;
// Family-1 long-bra rows stage the bra's D rows in LDS only while the
// workgroup's LDS stays within this (so the staging does not cost occupancy).
constexpr int DSTAGE_LDS_MAX = 40 * 1024;

// Persistent form of the batched builds (kern_persist.hip): the family-1
// 64-lane row tasks of the one- and two-root classes of every molecule in
// one launch over a queue of (descriptor, task) items.
bool persist_class(int li, int lj, int lk, int ll);
hipError_t launch_k1_persist(int pr, const BatchDesc *descs, const int32_t *items, int nitems, int *counter, size_t lds,
                             int grid, hipStream_t s);

// Indexed by class_id(li, lj, lk, ll); zero-initialised, filled by the
// static initialisers of the kernel units when the library loads.
extern ClassEntry g_classes[NCLS];

}  // namespace jk
