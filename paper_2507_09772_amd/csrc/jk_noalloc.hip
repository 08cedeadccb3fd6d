// jk_noalloc.hip -- jk_execute_noalloc (include/jk.h): the J/K build with
// its scratch in one fixed device array per GPU instead of plan-owned
// allocations, for callers that cannot allocate.
#include <hip/hip_runtime.h>

#include <mutex>

#include "jk_internal.h"

// The array is a device symbol: its host-side name is not a device address,
// so the address is looked up once per device (with that device current)
// and only that pointer is passed on.
static __device__ __align__(256) double scratch[JK_NOALLOC_SCRATCH_BYTES / sizeof(double)];
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[64];

static int noalloc_scratch(double **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(JK_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(JK_EDEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

extern "C" int jk_execute_noalloc(jk_plan *P, const double *D, int32_t nset, int32_t flags, int32_t precision,
                                  double mix_threshold, double omega, double *J, double *K, void *stream) {
    int rc = check_execute_args(P, D, nset, flags, precision, mix_threshold, omega, J, K);
    if (rc) return rc;
    // carve the array: J', K', Cartesian D, pair-ordered J', block maxima,
    // counters, each on a 256-byte boundary
    const ScratchSizes z = scratch_sizes(P, nset);
    const size_t parts[6] = {z.mat, z.mat, z.dc, z.jp, z.dmax, z.nsel};
    size_t off[6], need = 0;
    for (int k = 0; k < 6; ++k) {
        off[k] = need;
        need += (parts[k] + 31) / 32 * 32;  // elements of 8 bytes, rounded to 256 bytes
    }
    if (need * sizeof(double) > (size_t)JK_NOALLOC_SCRATCH_BYTES)
        return fail(JK_EINVAL, "build needs %zu bytes of scratch, the fixed array holds %zu", need * sizeof(double),
                    (size_t)JK_NOALLOC_SCRATCH_BYTES);
    double *base = nullptr;
    if ((rc = noalloc_scratch(&base))) return rc;
    Scratch sc{base + off[0], base + off[1], base + off[2], base + off[3], base + off[4],
               (unsigned long long *)(base + off[5])};
    return execute_impl(P, D, nset, flags, precision, mix_threshold, omega, J, K, (hipStream_t)stream, sc, false);
}

