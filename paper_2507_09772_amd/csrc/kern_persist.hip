// kern_persist.hip -- the persistent form of the batched builds for the
// one- and two-root classes (family 1, 64-lane row tasks): one launch walks
// a global queue of (descriptor, row task) items of every such class and
// molecule, heaviest first; each workgroup takes the next item with one
// atomic and runs it with the class's row-task body.
#include "jk_registry.h"

namespace jk {

// Classes of the persistent kernel: total angular momentum <= 3 (one or
// two roots), in a fixed order.
#define JK_PERSIST_CLASSES(X) \
    X(0, 0, 0, 0) X(1, 0, 0, 0) X(1, 0, 1, 0) X(1, 1, 0, 0) X(2, 0, 0, 0) X(1, 1, 1, 0) X(2, 0, 1, 0) X(2, 1, 0, 0) X(3, 0, 0, 0)

bool persist_class(int li, int lj, int lk, int ll) {
#define JK_PC(a, b, c, d) if (li == a && lj == b && lk == c && ll == d) return true;
    JK_PERSIST_CLASSES(JK_PC)
#undef JK_PC
    return false;
}

// items: [nitems][2] (descriptor, task); counter starts at 0 each build.
template <typename R>
__global__ void __launch_bounds__(64) jk_k1_persist(const BatchDesc *__restrict__ descs, const int32_t *__restrict__ items,
                                                    int nitems, int *counter) {
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = next;
        __syncthreads();
        if (it >= nitems) break;  // uniform in the workgroup: every wave ends
        const int di = __builtin_amdgcn_readfirstlane(items[2 * it]);
        const int task = __builtin_amdgcn_readfirstlane(items[2 * it + 1]);
        const JkArgs a = descs[di].a;
        const int cid = __builtin_amdgcn_readfirstlane(descs[di].pad[0]);
        switch (cid) {
#define JK_PC(A, B, C, D)                                  \
    case class_id(A, B, C, D):                             \
        k1_row_task<A, B, C, D, R, 64>(a, task);           \
        break;
            JK_PERSIST_CLASSES(JK_PC)
#undef JK_PC
            default:
                break;
        }
        __syncthreads();  // the next item reuses the LDS rows
    }
}

hipError_t launch_k1_persist(int pr, const BatchDesc *descs, const int32_t *items, int nitems, int *counter, size_t lds,
                             int grid, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (lds > (size_t)ROW_LDS_MAX) return hipErrorInvalidValue;
    static bool opted[2] = {false, false};
    if (lds > 64 * 1024 && !opted[pr]) {
        const hipError_t e = pr ? hipFuncSetAttribute((const void *)&jk_k1_persist<float>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, ROW_LDS_MAX)
                                : hipFuncSetAttribute((const void *)&jk_k1_persist<double>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, ROW_LDS_MAX);
        if (e != hipSuccess) return e;
        opted[pr] = true;
    }
    if (pr) hipLaunchKernelGGL((jk_k1_persist<float>), dim3(grid), dim3(64), lds, s, descs, items, nitems, counter);
    else hipLaunchKernelGGL((jk_k1_persist<double>), dim3(grid), dim3(64), lds, s, descs, items, nitems, counter);
    return hipGetLastError();
}

}  // namespace jk
