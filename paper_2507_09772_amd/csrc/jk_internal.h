// jk_internal.h -- host-side plan structures shared by the planner
// (jk_api.hip) and the batched builds (jk_batch.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/jk.h"
#include "jk_registry.h"

using namespace jk;

// Error reporting: fail() stores a thread-local message and returns code.
extern thread_local std::string g_err;
int fail(int code, const char *fmt, ...);

#define HIPCHK(expr)                                                                   \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(e_ == hipErrorOutOfMemory ? JK_ENOMEM : JK_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);             \
    } while (0)

struct ShellDev {
    const int32_t *l, *nprim, *poff, *atom;
    const double *exps, *coefs, *coords;
};

struct AoMaps {
    const int32_t *sh_c, *comp_c;  // Cartesian AO -> shell, component
    const int32_t *sh_e, *comp_e;  // external AO -> shell, component
    const int32_t *l, *aoc, *aoe;  // per shell
    const double *c2s;             // concatenated T_l, rows m, cols Cartesian
};

// ---------------------------------------------------------------------------
// element functions of the basis transforms, shared by the single and the
// batched builds
// ---------------------------------------------------------------------------
// Adds the pair-ordered J' buffer into the Cartesian J' (after the class
// kernels): t = ((s * npair) + p) * 64 + lane; the lanes of one pair walk its
// elements.  Pairs own disjoint blocks (rows of the first shell, columns of
// the second), so plain adds suffice.
__device__ __forceinline__ void jp_scatter_elem(const PairRec *__restrict__ pairs, const int32_t *__restrict__ lsh,
                                                const double *__restrict__ jp, int64_t jpstride, double *Jc,
                                                int64_t mstride, int naoc, int npair, int64_t t) {
    const int e0 = (int)(t & 63);
    const int64_t u = t >> 6;
    const int p = (int)(u % npair);
    const int64_t s = u / npair;
    const PairRec &r = pairs[p];
    const int nb = ncart(lsh[r.jsh]), nab = ncart(lsh[r.ish]) * nb;
    for (int e = e0; e < nab; e += 64) {
        const double v = jp[s * jpstride + r.jp_off + (int64_t)e * r.pp_stride];
        if (v != 0.0) Jc[s * mstride + (int64_t)(r.aoi + e / nb) * naoc + r.aoj + e % nb] += v;
    }
}

__device__ __forceinline__ const double *c2s_of(const AoMaps &m, int l) {
    return m.c2s + (l == 0 ? jkt_c2s_offset[0] : l == 1 ? jkt_c2s_offset[1] : l == 2 ? jkt_c2s_offset[2]
                    : l == 3 ? jkt_c2s_offset[3] : jkt_c2s_offset[4]);
}

// Element t = (s, a, b) of Dc[s] = T^T D[s] T over the block-diagonal
// spherical-to-Cartesian map T.
__device__ __forceinline__ double sph_to_cart_elem(const AoMaps &m, const double *D, int nao, int naoc, int64_t t) {
    const int s = (int)(t / ((int64_t)naoc * naoc));
    const int a = (int)((t / naoc) % naoc), b = (int)(t % naoc);
    const int I = m.sh_c[a], J = m.sh_c[b];
    const int li = m.l[I], lj = m.l[J];
    const int ca = m.comp_c[a], cb = m.comp_c[b];
    const double *Ti = c2s_of(m, li), *Tj = c2s_of(m, lj);
    const int nci = ncart(li), ncj = ncart(lj);
    const double *Ds = D + (int64_t)s * nao * nao;
    double acc = 0.0;
    for (int i = 0; i < 2 * li + 1; ++i) {
        const double ti = Ti[i * nci + ca];
        if (ti == 0.0) continue;
        double r = 0.0;
        for (int j = 0; j < 2 * lj + 1; ++j) r += Ds[(int64_t)(m.aoe[I] + i) * nao + m.aoe[J] + j] * Tj[j * ncj + cb];
        acc += ti * r;
    }
    return acc;
}

// Element t = (s, i, j) of T (X + X^T) T^T (spherical) or X + X^T.
__device__ __forceinline__ double finalize_elem(const AoMaps &m, const double *X, int nao, int naoc, int spherical,
                                                int64_t t) {
    const int s = (int)(t / ((int64_t)nao * nao));
    const int i = (int)((t / nao) % nao), j = (int)(t % nao);
    const double *Xs = X + (int64_t)s * naoc * naoc;
    if (!spherical) return Xs[(int64_t)i * naoc + j] + Xs[(int64_t)j * naoc + i];
    const int I = m.sh_e[i], J = m.sh_e[j];
    const int li = m.l[I], lj = m.l[J];
    const int mi = m.comp_e[i], mj = m.comp_e[j];
    const int nci = ncart(li), ncj = ncart(lj);
    const double *Ti = c2s_of(m, li) + mi * nci, *Tj = c2s_of(m, lj) + mj * ncj;
    double v = 0.0;
    for (int a = 0; a < nci; ++a) {
        if (Ti[a] == 0.0) continue;
        const int ga = m.aoc[I] + a;
        double r = 0.0;
        for (int b = 0; b < ncj; ++b) {
            const int gb = m.aoc[J] + b;
            r += (Xs[(int64_t)ga * naoc + gb] + Xs[(int64_t)gb * naoc + ga]) * Tj[b];
        }
        v += Ti[a] * r;
    }
    return v;
}

// Entry t = (I, J) of max_s max_{a in I, b in J} |Dc[s][a][b]|.
__device__ __forceinline__ double dmax_elem(const double *Dc, const int32_t *aoc, const int32_t *l, int ns, int naoc,
                                           int nset, int t) {
    const int I = t / ns, J = t % ns;
    double m = 0.0;
    for (int s = 0; s < nset; ++s)
        for (int a = 0; a < ncart(l[I]); ++a)
            for (int b = 0; b < ncart(l[J]); ++b)
                m = fmax(m, fabs(Dc[(int64_t)s * naoc * naoc + (int64_t)(aoc[I] + a) * naoc + aoc[J] + b]));
    return m;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
    template <typename T> T *as() const { return (T *)p; }
};

struct ClassTask {
    int li, lj, lk, ll;
    int bt, kt, same, npb, npk, nbra;
    // row mode: long bras (positions into d_bra / d_cnt) and the short rest
    int nrow = 0, nsbra = 0, nstiles[2] = {0, 0};
    int64_t nq_row = 0;  // quartets of the long bras
    int nrowc[3] = {0, 0, 0};                    // row tasks per family
    int32_t *d_rowc[3] = {nullptr, nullptr, nullptr};  // (list position, ket begin, ket end) per task
    std::vector<int32_t> h_rowc[3];              // host copies (batched builds)
    int nsrow = 0;                               // short bras as 64-lane row tasks
    int32_t *d_srowt = nullptr;
    std::vector<int32_t> h_srowt;
    int32_t *d_sbra = nullptr, *d_scnt = nullptr, *d_stile[2] = {nullptr, nullptr};
    int ncolK = 0, ncolL = 0, seg_same = 0;
    const int32_t *d_tshK = nullptr, *d_tshL = nullptr;
    int fam[2];          // family per precision (0 FP64, 1 FP32)
    bool split = true;   // mixed builds split this class by the bound (else all FP64)
    bool row_ok[2];      // row mode allowed per precision
    bool row_short[2];   // short bras in row mode too (64-lane workgroups)
    int ntiles[2];       // per family - 1
    int64_t nq, npq;
    double flops;
    int32_t *d_bra = nullptr, *d_cnt = nullptr, *d_tile[2] = {nullptr, nullptr};
    const int32_t *d_ket = nullptr;
};

struct jk_plan {
    int ns = 0, natom = 0, sph = 0, nao = 0, naoc = 0;
    double cutoff = 0.0;
    std::vector<int32_t> l, nprim, atom, poff, aoc, aoe;
    std::vector<int32_t> pair_of;  // [ns*ns] -> pair index
    std::vector<PairRec> hpairs;
    std::vector<double> Qsh;
    std::vector<ClassTask> cls;
    std::vector<void *> allocs;  // everything below is freed with the plan
    ShellDev sh{};
    PairRec *d_pairs = nullptr;
    PrimPair *d_pp = nullptr;
    AoMaps maps{};
    double *d_Jc = nullptr, *d_Kc = nullptr, *d_Dc = nullptr;
    int scratch_nset = 0, dc_nset = 0;
    double *d_jp = nullptr;  // pair-ordered J'_KL buffer [scratch_nset][njp]
    double *d_det = nullptr;  // JK_DETERMINISTIC limbs, 9 x det_len elements
    int64_t det_len = 0;
    int64_t njp = 0;
    // quartets evaluated per launch of the last build: [class][precision][kind]
    // counted on the device (NSEL_SLOTS counters each), or known on the host
    unsigned long long *d_nsel = nullptr;
    const unsigned long long *last_nsel = nullptr;  // device counters of the last build
    std::vector<int64_t> last_fixed;                 // host count per launch, -1: on the device
    int last_precision = -1;
    int32_t *d_tpos = nullptr;                         // shell -> index within its type
    double dscreen = 0.0;  // density screening threshold for later builds (0: off)
    bool no_row = false;  // JK_NO_ROW=1 in the environment: tiles only (A/B measurements)
    bool no_dstage = false;  // JK_NO_DSTAGE=1: family-1 rows read D from global memory (A/B measurements)
    double *d_dmax = nullptr;
    Tables tab{};
    jk_stats stats{};
    int device = 0;
    // class kernels of one build spread over the caller's stream and these
    // (JK_STREAMS, default 4 in all; default priority, non-blocking), forked
    // from and joined back into the caller's stream by events
    static constexpr int MAXSTREAM = 8;
    int nstream = 1;
    hipStream_t streams[MAXSTREAM] = {};
    hipEvent_t fork_ev = nullptr, join_ev[MAXSTREAM] = {};
    // per-kernel timing
    bool profile = false;
    std::vector<hipEvent_t> events;
    std::vector<jk_class_timing> timing;  // [(2 * class + (FP32 ? 1 : 0)) * 3 + kind]

    template <typename T>
    int alloc(T **p, size_t n) {
        if (n == 0) n = 1;
        hipError_t e = hipMalloc((void **)p, sizeof(T) * n);
        if (e != hipSuccess) return fail(e == hipErrorOutOfMemory ? JK_ENOMEM : JK_EDEVICE, "hipMalloc(%zu): %s", sizeof(T) * n, hipGetErrorString(e));
        allocs.push_back(*p);
        return 0;
    }
    template <typename T>
    int put(T **p, const std::vector<T> &v) {
        int rc = alloc(p, v.size());
        if (rc) return rc;
        if (!v.empty()) HIPCHK(hipMemcpy(*p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
        return 0;
    }
    ~jk_plan() {
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (int k = 1; k < nstream; ++k) {
            if (streams[k]) (void)hipStreamDestroy(streams[k]);
            if (join_ev[k]) (void)hipEventDestroy(join_ev[k]);
        }
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        for (void *p : allocs) (void)hipFree(p);
    }
};

// Device scratch of one build: Cartesian J', K' and density, the pair-ordered
// J'_KL buffer, the density block maxima and the per-launch counters.
struct Scratch {
    double *Jc, *Kc, *Dc, *jp, *dmax;
    unsigned long long *nsel;
    // JK_DETERMINISTIC: J', K' and the pair-ordered J' as integer limbs,
    // [3 buffers][3 limbs][detL] (null when the caller's scratch has none)
    double *det = nullptr;
    int64_t detL = 0;
};

// Elements of each scratch array for a build with nset densities.
struct ScratchSizes {
    size_t mat, jp, dc, dmax, nsel;
};
inline ScratchSizes scratch_sizes(const jk_plan *P, int nset) {
    ScratchSizes z;
    z.mat = (size_t)nset * P->naoc * P->naoc;
    z.jp = (size_t)nset * P->njp;
    z.dc = P->sph ? z.mat : 0;
    z.dmax = (size_t)P->ns * P->ns + 1;  // the table and its largest entry
    z.nsel = 8 * std::max<size_t>(P->cls.size(), 1) * NSEL_SLOTS * NSEL_STRIDE;
    return z;
}

// Argument checks shared by the build entry points (0 or a JK_E* code).
int check_execute_args(const jk_plan *P, const double *D, int32_t nset, int32_t flags, int32_t precision,
                       double mix_threshold, double omega, double *J, double *K);
// One J/K build into the given scratch (arguments already checked).
int execute_impl(jk_plan *P, const double *D, int32_t nset, int32_t flags, int32_t precision, double mix_threshold,
                 double omega, double *J, double *K, hipStream_t s, const Scratch &sc, bool allow_profile);
