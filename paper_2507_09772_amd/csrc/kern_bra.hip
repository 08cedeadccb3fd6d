// kern_bra.hip -- kernel instantiations for one bra angular pair (JK_LI, JK_LJ),
// compiled once per pair with -DJK_LI=.. -DJK_LJ=.. so the classes build in
// parallel.  Kets (LK, LL) run over every canonical pair with LK >= LL and
// (LK, LL) <= (JK_LI, JK_LJ) lexicographically.
#include "jk_registry.h"

#ifndef JK_LI
#error "JK_LI / JK_LJ must be defined"
#endif

namespace jk {

template <int LI, int LJ, int LK, int LL, typename R, int MODE>
static hipError_t launch_k1(const JkArgs &a, hipStream_t s) {
    int grid;
    if constexpr (MODE == MODE_JK) grid = (a.ntiles + 3) / 4;
    else grid = (a.nq + 255) / 256;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((jk_k1<LI, LJ, LK, LL, R, MODE>), dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

// Dynamic LDS above 64 KB needs a per-kernel opt-in (once per kernel).
template <typename K>
static hipError_t lds_opt_in(K kernel, size_t lds, bool &done) {
    if (lds <= 64 * 1024 || done) return hipSuccess;
    const hipError_t e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, ROW_LDS_MAX);
    if (e == hipSuccess) done = true;
    return e;
}

static size_t k1_row_lds(const JkArgs &a, int li, int lj) {
    const int ncols = a.ncolK + (a.seg_same ? 0 : a.ncolL);
    return sizeof(PrimPair) * (size_t)a.npb +
           sizeof(double) * a.nset * ((size_t)(ncart(li) + ncart(lj)) * ncols + (size_t)ncart(li) * ncart(lj)) +
           (a.dstage ? sizeof(double) * a.nset * (size_t)(ncart(li) + ncart(lj)) * ncols : 0);
}

template <int LI, int LJ, int LK, int LL, typename R, int NT>
static hipError_t launch_row(const JkArgs &a, hipStream_t s) {
    if (a.nrow <= 0) return hipSuccess;
    const size_t lds = k1_row_lds(a, LI, LJ);
    if (lds > (size_t)ROW_LDS_MAX) return hipErrorInvalidValue;
    static bool opted_in = false;
    const hipError_t e = lds_opt_in(&jk_k1_row<LI, LJ, LK, LL, R, NT, false>, lds, opted_in);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((jk_k1_row<LI, LJ, LK, LL, R, NT, false>), dim3(a.nrow), dim3(NT), lds, s, a,
                       (const BatchDesc *)nullptr, 0);
    return hipGetLastError();
}

template <int LI, int LJ, int LK, int LL, typename R, int NT>
static hipError_t launch_row2(const JkArgs &a, hipStream_t s) {
    if (a.nrow <= 0) return hipSuccess;
    using L = K2RowLds<LI, LJ, LK, LL>;
    const int ncols = a.ncolK + (a.seg_same ? 0 : a.ncolL);
    const size_t lds = (NT / 64) * L::template fixed<R>() + (size_t)a.nset * L::per_set(ncols);
    if (lds > (size_t)ROW_LDS_MAX) return hipErrorInvalidValue;
    static bool opted_in = false;
    const hipError_t e = lds_opt_in(&jk_k2_row<LI, LJ, LK, LL, R, NT, false>, lds, opted_in);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((jk_k2_row<LI, LJ, LK, LL, R, NT, false>), dim3(a.nrow), dim3(NT), lds, s, a,
                       (const BatchDesc *)nullptr, 0);
    return hipGetLastError();
}

template <int LI, int LJ, int LK, int LL, typename R, int NT>
static hipError_t launch_row3(const JkArgs &a, hipStream_t s) {
    if (a.nrow <= 0) return hipSuccess;
    using F = K3Cfg<LI, LJ, LK, LL>;
    const int ncols = a.ncolK + (a.seg_same ? 0 : a.ncolL);
    const size_t lds = (NT / 64) * F::template wave_bytes<R>() + (size_t)a.nset * F::per_set(ncols);
    if (lds > (size_t)ROW_LDS_MAX) return hipErrorInvalidValue;
    static bool opted_in = false;
    const hipError_t e = lds_opt_in(&jk_k3_row<LI, LJ, LK, LL, R, NT, false>, lds, opted_in);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((jk_k3_row<LI, LJ, LK, LL, R, NT, false>), dim3(a.nrow), dim3(NT), lds, s, a,
                       (const BatchDesc *)nullptr, 0);
    return hipGetLastError();
}

template <int LI, int LJ, int LK, int LL, typename R>
static hipError_t launch_row3_batch(const BatchDesc *d, int ndesc, int total, size_t lds, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    if (lds > (size_t)ROW_LDS_MAX) return hipErrorInvalidValue;
    static bool opted_in = false;
    const hipError_t e = lds_opt_in(&jk_k3_row<LI, LJ, LK, LL, R, 64, true>, lds, opted_in);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((jk_k3_row<LI, LJ, LK, LL, R, 64, true>), dim3(total), dim3(64), lds, s, JkArgs{}, d, ndesc);
    return hipGetLastError();
}

// Batched 64-lane row tasks; lds = the largest workgroup need over the descriptors.
template <int LI, int LJ, int LK, int LL, typename R>
static hipError_t launch_row_batch(const BatchDesc *d, int ndesc, int total, size_t lds, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    if (lds > (size_t)ROW_LDS_MAX) return hipErrorInvalidValue;
    static bool opted_in = false;
    const hipError_t e = lds_opt_in(&jk_k1_row<LI, LJ, LK, LL, R, 64, true>, lds, opted_in);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((jk_k1_row<LI, LJ, LK, LL, R, 64, true>), dim3(total), dim3(64), lds, s, JkArgs{}, d, ndesc);
    return hipGetLastError();
}

template <int LI, int LJ, int LK, int LL, typename R>
static hipError_t launch_row2_batch(const BatchDesc *d, int ndesc, int total, size_t lds, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    if (lds > (size_t)ROW_LDS_MAX) return hipErrorInvalidValue;
    static bool opted_in = false;
    const hipError_t e = lds_opt_in(&jk_k2_row<LI, LJ, LK, LL, R, 64, true>, lds, opted_in);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((jk_k2_row<LI, LJ, LK, LL, R, 64, true>), dim3(total), dim3(64), lds, s, JkArgs{}, d, ndesc);
    return hipGetLastError();
}

template <int LI, int LJ, int LK, int LL, typename R, int MODE>
static hipError_t launch_k2(const JkArgs &a, hipStream_t s) {
    constexpr int QW = k2_qw(LI, LJ, LK, LL);
    int grid;
    if constexpr (MODE == MODE_JK) grid = a.ntiles;
    else grid = (a.nq + QW - 1) / QW;
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((jk_k2<LI, LJ, LK, LL, R, MODE>), dim3(grid), dim3(64), 0, s, a);
    return hipGetLastError();
}

// Batched tiles: one wave (family 1) or one workgroup (family 2) per tile.
template <int LI, int LJ, int LK, int LL, typename R>
static hipError_t launch_k1_batch(const BatchDesc *d, int ndesc, int total, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((jk_k1_batch<LI, LJ, LK, LL, R>), dim3((total + 3) / 4), dim3(256), 0, s, d, ndesc, total);
    return hipGetLastError();
}

template <int LI, int LJ, int LK, int LL, typename R>
static hipError_t launch_k2_batch(const BatchDesc *d, int ndesc, int total, hipStream_t s) {
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL((jk_k2_batch<LI, LJ, LK, LL, R>), dim3(total), dim3(64), 0, s, d, ndesc, total);
    return hipGetLastError();
}

// Classes with a g shell (l = 4) get the single-molecule kernels only (no
// 64-lane short-bra row kernels and no batched kernels), which keeps their
// compile time in bounds: short bras run as tiles, and batched builds of
// such molecules report JK_EUNSUPPORTED.
template <int LK, int LL>
static void reg_one() {
    constexpr int LI = JK_LI, LJ = JK_LJ;
    constexpr bool FULL = LI < 4;
    if constexpr (LK >= LL && (LK < LI || (LK == LI && LL <= LJ))) {
        ClassEntry &e = g_classes[class_id(LI, LJ, LK, LL)];
        if constexpr (has_family1(LI, LJ, LK, LL)) {
            e.tiles[0][0] = &launch_k1<LI, LJ, LK, LL, double, MODE_JK>;
            e.tiles[0][1] = &launch_k1<LI, LJ, LK, LL, float, MODE_JK>;
            e.row[0][0] = &launch_row<LI, LJ, LK, LL, double, 256>;
            e.row[0][1] = &launch_row<LI, LJ, LK, LL, float, 256>;
            if constexpr (FULL) {
                e.srow[0][0] = &launch_row<LI, LJ, LK, LL, double, 64>;
                e.srow[0][1] = &launch_row<LI, LJ, LK, LL, float, 64>;
                e.batch_row[0][0] = &launch_row_batch<LI, LJ, LK, LL, double>;
                e.batch_row[0][1] = &launch_row_batch<LI, LJ, LK, LL, float>;
                e.batch[0][0] = &launch_k1_batch<LI, LJ, LK, LL, double>;
                e.batch[0][1] = &launch_k1_batch<LI, LJ, LK, LL, float>;
            }
        }
        if constexpr (has_family2(LI, LJ, LK, LL)) {
            e.tiles[1][0] = &launch_k2<LI, LJ, LK, LL, double, MODE_JK>;
            e.tiles[1][1] = &launch_k2<LI, LJ, LK, LL, float, MODE_JK>;
            e.row[1][0] = &launch_row2<LI, LJ, LK, LL, double, 256>;
            e.row[1][1] = &launch_row2<LI, LJ, LK, LL, float, 256>;
            if constexpr (FULL) {
                e.srow[1][0] = &launch_row2<LI, LJ, LK, LL, double, 64>;
                e.srow[1][1] = &launch_row2<LI, LJ, LK, LL, float, 64>;
                e.batch_row[1][0] = &launch_row2_batch<LI, LJ, LK, LL, double>;
                e.batch_row[1][1] = &launch_row2_batch<LI, LJ, LK, LL, float>;
            }
            e.row_fixed[1][0] = K2RowLds<LI, LJ, LK, LL>::template fixed<double>();
            e.row_fixed[1][1] = K2RowLds<LI, LJ, LK, LL>::template fixed<float>();
            if constexpr (FULL) {
                e.batch[1][0] = &launch_k2_batch<LI, LJ, LK, LL, double>;
                e.batch[1][1] = &launch_k2_batch<LI, LJ, LK, LL, float>;
            }
        }
        if constexpr (has_family3(LI, LJ, LK, LL)) {
            e.row[2][0] = &launch_row3<LI, LJ, LK, LL, double, 256>;
            e.row[2][1] = &launch_row3<LI, LJ, LK, LL, float, 256>;
            if constexpr (FULL) {
                e.srow[2][0] = &launch_row3<LI, LJ, LK, LL, double, 64>;
                e.srow[2][1] = &launch_row3<LI, LJ, LK, LL, float, 64>;
                e.batch_row[2][0] = &launch_row3_batch<LI, LJ, LK, LL, double>;
                e.batch_row[2][1] = &launch_row3_batch<LI, LJ, LK, LL, float>;
            }
            e.row_fixed[2][0] = K3Cfg<LI, LJ, LK, LL>::template wave_bytes<double>();
            e.row_fixed[2][1] = K3Cfg<LI, LJ, LK, LL>::template wave_bytes<float>();
        }
        if constexpr (default_family(LI, LJ, LK, LL) == 1) {
            e.ex64 = &launch_k1<LI, LJ, LK, LL, double, MODE_EXPORT>;
            e.ex32 = &launch_k1<LI, LJ, LK, LL, float, MODE_EXPORT>;
        } else {
            e.ex64 = &launch_k2<LI, LJ, LK, LL, double, MODE_EXPORT>;
            e.ex32 = &launch_k2<LI, LJ, LK, LL, float, MODE_EXPORT>;
        }
    }
}

static int reg_all() {
    reg_one<0, 0>();
    reg_one<1, 0>(); reg_one<1, 1>();
    reg_one<2, 0>(); reg_one<2, 1>(); reg_one<2, 2>();
    reg_one<3, 0>(); reg_one<3, 1>(); reg_one<3, 2>(); reg_one<3, 3>();
    reg_one<4, 0>(); reg_one<4, 1>(); reg_one<4, 2>(); reg_one<4, 3>(); reg_one<4, 4>();
    return 0;
}

static const int registered = reg_all();

}  // namespace jk
