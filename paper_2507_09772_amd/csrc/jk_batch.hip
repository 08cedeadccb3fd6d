// jk_batch.hip -- batched J/K builds over many molecules (jk_batch_* in
// include/jk.h).
//
// Every molecule keeps its own plan (pairs, sorted ket lists, tiles).  The
// batch gathers, per angular class and kernel family, the class tasks of all
// molecules into one descriptor array; one launch per group covers the
// tiles of all its descriptors, heaviest molecule first.  The
// basis transforms, clearing and finalisation run as batched kernels with
// one grid row per molecule.  The whole sequence is recorded once into a
// hipGraph and replayed on every call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <tuple>
#include <vector>

#include "jk_internal.h"

namespace {

// Per-molecule view for the batched helper kernels (device copy).
struct MolDesc {
    AoMaps maps;
    const double *D;         // caller's density [nset][nao][nao]
    double *J, *K;           // caller's outputs
    double *Dc, *Jc, *Kc;    // batch scratch [nset][naoc][naoc]
    double *jp;              // pair-ordered J'_KL [nset][njp]
    const PairRec *pairs;
    int64_t njp;
    double *dmax;            // [ns][ns]
    int32_t nao, naoc, ns, sph, npair;
};

// Dc = Cartesian density (transformed or copied); Jc = Kc = 0.
__global__ void kb_prepare(const MolDesc *mols, int nset) {
    const MolDesc &m = mols[blockIdx.y];
    const int64_t tot = (int64_t)nset * m.naoc * m.naoc;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        m.Dc[t] = m.sph ? sph_to_cart_elem(m.maps, m.D, m.nao, m.naoc, t) : m.D[t];
        m.Jc[t] = 0.0;
        m.Kc[t] = 0.0;
    }
    const int64_t njp = (int64_t)nset * m.njp;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < njp; t += (int64_t)gridDim.x * blockDim.x)
        m.jp[t] = 0.0;
}

__global__ void kb_jp_scatter(const MolDesc *mols, int nset) {
    const MolDesc &m = mols[blockIdx.y];
    const int64_t nt = (int64_t)nset * m.npair * 64;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x)
        jp_scatter_elem(m.pairs, m.maps.l, m.jp, m.njp, m.Jc, (int64_t)m.naoc * m.naoc, m.naoc, m.npair, t);
}

__global__ void kb_dmax(const MolDesc *mols, int nset) {
    const MolDesc &m = mols[blockIdx.y];
    const int tot = m.ns * m.ns;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += gridDim.x * blockDim.x)
        m.dmax[t] = dmax_elem(m.Dc, m.maps.aoc, m.maps.l, m.ns, m.naoc, nset, t);
}

// m.dmax[ns * ns] = the largest entry of molecule m's table (one workgroup each).
__global__ void __launch_bounds__(256) kb_dmax_all(const MolDesc *mols) {
    const MolDesc &m = mols[blockIdx.x];
    __shared__ double part[256];
    double v = 0.0;
    for (int t = threadIdx.x; t < m.ns * m.ns; t += 256) v = fmax(v, m.dmax[t]);
    part[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] = fmax(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) m.dmax[m.ns * m.ns] = part[0];
}

__global__ void kb_finalize(const MolDesc *mols, int nset) {
    const MolDesc &m = mols[blockIdx.y];
    const int64_t tot = (int64_t)nset * m.nao * m.nao;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        m.J[t] = finalize_elem(m.maps, m.Jc, m.nao, m.naoc, m.sph, t);
        m.K[t] = finalize_elem(m.maps, m.Kc, m.nao, m.naoc, m.sph, t);
    }
}

__global__ void kb_zero_i32(int *p, int n) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) p[t] = 0;
}

__global__ void kb_zero_u64(unsigned long long *p, int n) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) p[t] = 0ull;
}

// One launch: the descriptors [first, first + count) of one (class, family)
// group.
struct Group {
    int cid, fam;
    int pr, sel;       // kernel precision (0 FP64, 1 FP32); quartet selection (SEL_*)
    int kind;          // 0: tiles, 1: 64-lane row tasks
    size_t lds;        // row tasks: largest dynamic LDS over the descriptors
    int first, count;
    int total_tiles;
    double work;       // model FLOPs of the group, for launch order
};

}  // namespace

struct jk_batch {
    std::vector<jk_plan *> plans;
    int nmol = 0, nset = 0, precision = 0, device = 0;
    double thr = 0.0;
    std::vector<MolDesc> hmol;
    MolDesc *d_mol = nullptr;
    std::vector<BatchDesc> hdesc;
    BatchDesc *d_desc = nullptr;
    std::vector<Group> groups;
    unsigned long long *d_ctr = nullptr;  // evaluated quartets per descriptor (NSEL_SLOTS counters each)
    // persistent form: per precision, the (descriptor, task) queue of the
    // one- and two-root family-1 row tasks, its length, LDS and grid
    struct Persist {
        int32_t *items = nullptr;
        int nitems = 0;
        size_t lds = 0;
        int grid = 0;
    } persist[2];
    int *d_pctr = nullptr;  // queue heads, one per precision
    std::vector<int64_t> fixed;           // per descriptor: its quartet count when not counted on the device
    std::vector<int> dprec;               // per descriptor: kernel precision (0 FP64, 1 FP32)
    int32_t *d_tasks = nullptr;  // row tasks of the row-kind descriptors
    int nctr = 0;
    int64_t max_elems = 0;      // largest nset * naoc^2 over the molecules
    int64_t max_jpt = 0;        // largest nset * npair * 64 (scatter threads)
    int max_ns2 = 0;
    std::vector<void *> allocs;
    MolDesc *h_stage = nullptr;  // pinned staging for pointer updates
    hipEvent_t stage_ev = nullptr;
    hipStream_t cap = nullptr;
    // class launches are independent (they only add into J', K' and the
    // pair-ordered J'): the graph holds them as nbranch parallel branches
    static constexpr int MAXBRANCH = 8;
    int nbranch = 1;
    hipStream_t branch[MAXBRANCH] = {};
    hipEvent_t fork = nullptr, join[MAXBRANCH] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    template <typename T>
    int alloc(T **p, size_t n) {
        if (n == 0) n = 1;
        const hipError_t e = hipMalloc((void **)p, sizeof(T) * n);
        if (e != hipSuccess)
            return fail(e == hipErrorOutOfMemory ? JK_ENOMEM : JK_EDEVICE, "hipMalloc(%zu): %s", sizeof(T) * n,
                        hipGetErrorString(e));
        allocs.push_back(*p);
        return 0;
    }
    ~jk_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        for (int k = 1; k < MAXBRANCH; ++k) {  // branch[0] is cap
            if (branch[k]) (void)hipStreamDestroy(branch[k]);
            if (join[k]) (void)hipEventDestroy(join[k]);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (stage_ev) (void)hipEventDestroy(stage_ev);
        if (h_stage) (void)hipHostFree(h_stage);
        for (void *p : allocs) (void)hipFree(p);
    }
};

static int grid_rows(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024)); }

// Records the whole batch build on b->cap.
static int record(jk_batch *b) {
    const int nm = b->nmol;
    hipStream_t s = b->cap;
    hipLaunchKernelGGL(kb_zero_u64, dim3(grid_rows(b->nctr)), dim3(256), 0, s, b->d_ctr, b->nctr);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(kb_prepare, dim3(grid_rows(b->max_elems), nm), dim3(256), 0, s, b->d_mol, b->nset);
    HIPCHK(hipGetLastError());
    if (b->precision == JK_MIXED) {
        hipLaunchKernelGGL(kb_dmax, dim3(grid_rows(b->max_ns2), nm), dim3(256), 0, s, b->d_mol, b->nset);
        hipLaunchKernelGGL(kb_dmax_all, dim3(nm), dim3(256), 0, s, b->d_mol);
        HIPCHK(hipGetLastError());
    }
    // fork: the class launches go round-robin (heaviest first) onto the
    // branch streams, which join before the scatter and finalisation
    HIPCHK(hipEventRecord(b->fork, s));
    for (int k = 1; k < b->nbranch; ++k) HIPCHK(hipStreamWaitEvent(b->branch[k], b->fork, 0));
    if (b->d_pctr) {
        hipLaunchKernelGGL(kb_zero_i32, dim3(1), dim3(64), 0, s, b->d_pctr, 2);
        HIPCHK(hipGetLastError());
    }
    int br = 0;
    for (int pr = 0; pr < 2; ++pr) {
        const jk_batch::Persist &q = b->persist[pr];
        if (q.nitems > 0)
            HIPCHK(launch_k1_persist(pr, b->d_desc, q.items, q.nitems, b->d_pctr + pr, q.lds, q.grid,
                                     b->branch[br++ % b->nbranch]));
    }
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const Group &g = b->groups[gi];
        const ClassEntry &e = g_classes[g.cid];
        hipStream_t bs = b->branch[(br + gi) % b->nbranch];
        if (g.kind == 1) HIPCHK(e.batch_row[g.fam - 1][g.pr](b->d_desc + g.first, g.count, g.total_tiles, g.lds, bs));
        else HIPCHK(e.batch[g.fam - 1][g.pr](b->d_desc + g.first, g.count, g.total_tiles, bs));
    }
    for (int k = 1; k < b->nbranch; ++k) {
        HIPCHK(hipEventRecord(b->join[k], b->branch[k]));
        HIPCHK(hipStreamWaitEvent(s, b->join[k], 0));
    }
    hipLaunchKernelGGL(kb_jp_scatter, dim3(grid_rows(b->max_jpt), nm), dim3(256), 0, s, b->d_mol, b->nset);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(kb_finalize, dim3(grid_rows(b->max_elems), nm), dim3(256), 0, s, b->d_mol, b->nset);
    HIPCHK(hipGetLastError());
    return 0;
}

extern "C" int jk_batch_create(jk_plan *const *plans, int32_t nmol, int32_t nset, int32_t precision,
                               double mix_threshold, jk_batch **out) {
    if (!out) return fail(JK_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plans || nmol < 1 || nmol > 65535) return fail(JK_EINVAL, "need 1 <= nmol <= 65535 plans");
    if (nset < 1) return fail(JK_EINVAL, "nset must be >= 1");
    if (precision != JK_FP64 && precision != JK_MIXED && precision != JK_FP32)
        return fail(JK_EINVAL, "bad precision %d", precision);
    if (precision == JK_MIXED && !(std::isfinite(mix_threshold) && mix_threshold >= 0.0))
        return fail(JK_EINVAL, "mix_threshold must be finite and >= 0");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    for (int m = 0; m < nmol; ++m) {
        if (!plans[m]) return fail(JK_EINVAL, "plans[%d] is NULL", m);
        if (plans[m]->device != dev) return fail(JK_EINVAL, "plans[%d] lives on device %d, current is %d", m, plans[m]->device, dev);
    }
    std::unique_ptr<jk_batch> b(new jk_batch);
    b->plans.assign(plans, plans + nmol);
    b->nmol = nmol;
    b->nset = nset;
    b->precision = precision;
    b->thr = mix_threshold;
    b->device = dev;
    int rc;

    // per-molecule scratch, one allocation each kind
    std::vector<int64_t> eoff(nmol + 1, 0), soff(nmol + 1, 0), joff(nmol + 1, 0);
    for (int m = 0; m < nmol; ++m) {
        const jk_plan *P = plans[m];
        const int64_t e = (int64_t)nset * P->naoc * P->naoc;
        eoff[m + 1] = eoff[m] + e;
        joff[m + 1] = joff[m] + (int64_t)nset * P->njp;
        b->max_jpt = std::max(b->max_jpt, (int64_t)nset * (int64_t)P->hpairs.size() * 64);
        soff[m + 1] = soff[m] + (int64_t)P->ns * P->ns + 1;  // the table and its largest entry
        b->max_elems = std::max(b->max_elems, e);
        b->max_ns2 = std::max(b->max_ns2, P->ns * P->ns);
    }
    double *Dc, *Jc, *Kc, *jp;
    double *dmax = nullptr;
    if ((rc = b->alloc(&Dc, eoff[nmol])) || (rc = b->alloc(&Jc, eoff[nmol])) || (rc = b->alloc(&Kc, eoff[nmol])) ||
        (rc = b->alloc(&jp, joff[nmol])))
        return rc;
    if (precision == JK_MIXED && (rc = b->alloc(&dmax, soff[nmol]))) return rc;

    // descriptors grouped by (class, family, kind, precision, selection);
    // heavy molecules first.  Unless row mode is off for the class, every
    // bra runs as 64-lane row tasks (K rows in LDS): the small molecules of
    // a batch have few long bras, and per-quartet K atomics would dominate.
    // Mixed precision: two descriptors per (molecule, class), the
    // single-precision pass over the quartets below the threshold and the
    // double-precision pass over the rest.
    using Key = std::tuple<int, int, int, int, int>;  // class, family, kind, precision, selection
    std::map<Key, std::vector<std::pair<double, BatchDesc>>> byg;
    std::vector<int32_t> alltasks;
    std::map<Key, size_t> glds;
    b->hmol.resize(nmol);
    for (int m = 0; m < nmol; ++m) {
        const jk_plan *P = plans[m];
        MolDesc &md = b->hmol[m];
        md.maps = P->maps;
        md.D = nullptr;
        md.J = md.K = nullptr;
        md.Dc = Dc + eoff[m];
        md.Jc = Jc + eoff[m];
        md.Kc = Kc + eoff[m];
        md.jp = jp + joff[m];
        md.pairs = P->d_pairs;
        md.njp = P->njp;
        md.npair = (int32_t)P->hpairs.size();
        md.dmax = dmax ? dmax + soff[m] : nullptr;
        md.nao = P->nao;
        md.naoc = P->naoc;
        md.ns = P->ns;
        md.sph = P->sph;
        for (size_t ci = 0; ci < P->cls.size(); ++ci) {
            const ClassTask &c = P->cls[ci];
            const bool msplit = precision == JK_MIXED && c.split;  // (else the class runs in FP64)
            const int npass = msplit ? 2 : 1;
            for (int pass = 0; pass < npass; ++pass) {
                const int pr = msplit ? (pass == 0 ? 1 : 0) : (precision == JK_FP32 ? 1 : 0);
                const int sel = msplit ? (pass == 0 ? SEL_LO : SEL_HI) : SEL_ALL;
                int f = c.fam[pr];
                const ClassEntry &ce = g_classes[class_id(c.li, c.lj, c.lk, c.ll)];
                const int ncols = c.ncolK + (c.seg_same ? 0 : c.ncolL);
                const size_t lds1 = row_lds_bytes(ce, f, pr, c.li, c.lj, nset, ncols, 1, c.npb);
                const int kind = c.row_ok[pr] && ce.batch_row[f - 1][pr] && lds1 <= (size_t)ROW_LDS_MAX ? 1 : 0;
                // tiles of a family-3 class run in its fallback family
                if (kind == 0 && f == 3) f = tile_fallback(c.li, c.lj, c.lk, c.ll);
                if (c.nq <= 0) continue;
                BatchDesc d{};
                JkArgs &a = d.a;
                a.pairs = P->d_pairs;
                a.pp = P->d_pp;
                a.bra_list = c.d_bra;
                a.bra_cnt = c.d_cnt;
                a.nbra = c.nbra;
                if (kind == 0) {  // (f <= 2 here)
                    a.tile_off = c.d_tile[f - 1];
                    a.ntiles = c.ntiles[f - 1];
                }
                a.ket_list = c.d_ket;
                a.same = c.same;
                a.npb = c.npb;
                a.npk = c.npk;
                a.nq = (int32_t)c.nq;
                a.tpos = P->d_tpos;
                a.aoc = P->maps.aoc;
                a.D = md.Dc;
                a.J = md.Jc;
                a.K = md.Kc;
                a.mstride = (int64_t)P->naoc * P->naoc;
                a.jp = md.jp;
                a.jpstride = P->njp;
                a.nao = P->naoc;
                a.nset = nset;
                a.do_j = 1;
                a.do_k = 1;
                a.dmax = md.dmax;
                a.nshell = P->ns;
                a.sel = sel;
                a.mix_thr = mix_threshold;
                a.tab = P->tab;
                d.pad[1] = a.ntiles;  // work units (tiles or row tasks)
                if (kind == 1) {
                    // every bra of the class: long bras in chunks, short ones whole
                    const size_t first = alltasks.size();
                    alltasks.insert(alltasks.end(), c.h_rowc[f - 1].begin(), c.h_rowc[f - 1].end());
                    alltasks.insert(alltasks.end(), c.h_srowt.begin(), c.h_srowt.end());
                    d.pad[1] = (int32_t)((alltasks.size() - first) / 3);
                    d.pad[2] = (int32_t)first;  // offset into the task buffer (host only)
                    a.nrow = d.pad[1];
                    a.tshK = c.d_tshK;
                    a.tshL = c.d_tshL;
                    a.ncolK = c.ncolK;
                    a.ncolL = c.ncolL;
                    a.seg_same = c.seg_same;
                    if (alltasks.size() > (size_t)INT32_MAX) return fail(JK_EINVAL, "too many row tasks");
                }
                if (!(kind == 1 || ce.batch[f - 1][pr]))
                    return fail(JK_EUNSUPPORTED, "class (%d%d|%d%d) has no batched kernel", c.li, c.lj, c.lk, c.ll);
                const Key key = std::make_tuple(class_id(c.li, c.lj, c.lk, c.ll), f, kind, pr, sel);
                byg[key].push_back({c.flops, d});
                if (kind == 1) glds[key] = std::max(glds[key], lds1);
            }
        }
    }
    std::vector<int32_t> hdesc_tasks;  // work units per descriptor
    std::vector<double> dwork;         // model FLOPs per descriptor
    std::vector<int32_t> dclass;       // class id per descriptor
    for (auto &kv : byg) {
        auto &v = kv.second;
        std::stable_sort(v.begin(), v.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
        Group g{};
        g.cid = std::get<0>(kv.first);
        g.fam = std::get<1>(kv.first);
        g.kind = std::get<2>(kv.first);
        g.pr = std::get<3>(kv.first);
        g.sel = std::get<4>(kv.first);
        g.lds = g.kind == 1 ? glds[kv.first] : 0;
        g.first = (int)b->hdesc.size();
        g.count = (int)v.size();
        int64_t tiles = 0;
        for (auto &x : v) {
            x.second.tile_base = (int32_t)tiles;
            tiles += x.second.pad[1];
            g.work += x.first;
            hdesc_tasks.push_back(x.second.pad[1]);
            dwork.push_back(x.first);
            dclass.push_back(g.cid);
            b->dprec.push_back(g.pr);
            b->hdesc.push_back(x.second);
        }
        if (tiles > INT32_MAX) return fail(JK_EINVAL, "too many tiles in one class group");
        g.total_tiles = (int)tiles;
        b->groups.push_back(g);
    }
    std::stable_sort(b->groups.begin(), b->groups.end(), [](const Group &x, const Group &y) { return x.work > y.work; });
    // row tasks to the device
    if ((rc = b->alloc(&b->d_tasks, alltasks.size()))) return rc;
    if (!alltasks.empty())
        HIPCHK(hipMemcpy(b->d_tasks, alltasks.data(), sizeof(int32_t) * alltasks.size(), hipMemcpyHostToDevice));
    for (size_t gi = 0; gi < b->groups.size(); ++gi) {
        const Group &g = b->groups[gi];
        for (int k = 0; k < g.count; ++k) {
            BatchDesc &d = b->hdesc[g.first + k];
            if (g.kind == 1) d.a.row_pos = b->d_tasks + d.pad[2];
        }
    }
    // persistent form (JK_BATCH_PERSIST=1; off by default: measured slower
    // than the per-class launches on parallel branches): the family-1 row
    // tasks of the one- and two-root classes leave their per-class launches
    // for one queue per precision, ordered by work per task (heaviest first)
    std::vector<std::vector<std::pair<double, std::pair<int32_t, int32_t>>>> pitems(2);
    {
        const char *pe = getenv("JK_BATCH_PERSIST");
        const bool on = pe && pe[0] == '1';
        std::vector<Group> keep;
        for (const Group &g : b->groups) {
            const int li = g.cid / 125, lj = (g.cid / 25) % 5, lk = (g.cid / 5) % 5, ll = g.cid % 5;
            if (!(on && g.kind == 1 && g.fam == 1 && persist_class(li, lj, lk, ll))) {
                keep.push_back(g);
                continue;
            }
            for (int k = 0; k < g.count; ++k) {
                const int di = g.first + k;
                const int ntask = hdesc_tasks[di];
                const double w = dwork[di] / std::max(ntask, 1);
                for (int t = 0; t < ntask; ++t) pitems[g.pr].push_back({w, {di, t}});
            }
            b->persist[g.pr].lds = std::max(b->persist[g.pr].lds, g.lds);
        }
        b->groups = keep;
    }
    // evaluated-quartet counters per descriptor (mixed precision only: with
    // every quartet selected the count is the descriptor's)
    const size_t per = (size_t)NSEL_SLOTS * NSEL_STRIDE;
    b->nctr = (int)(std::max<size_t>(b->hdesc.size(), 1) * per);
    if ((rc = b->alloc(&b->d_ctr, b->nctr))) return rc;
    b->fixed.assign(b->hdesc.size(), -1);
    for (size_t k = 0; k < b->hdesc.size(); ++k) {
        BatchDesc &d = b->hdesc[k];
        if (precision == JK_MIXED) {
            d.a.nsel = b->d_ctr + k * per;
        } else {
            d.a.nsel = nullptr;
            b->fixed[k] = d.a.nq;
        }
        d.pad[0] = dclass[k];  // the class (the persistent kernel's switch)
        d.pad[1] = d.pad[2] = 0;
    }
    if ((rc = b->alloc(&b->d_desc, b->hdesc.size())) || (rc = b->alloc(&b->d_mol, nmol))) return rc;
    int ncu = 0;
    HIPCHK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    for (int pr = 0; pr < 2; ++pr) {
        auto &v = pitems[pr];
        if (v.empty()) continue;
        std::stable_sort(v.begin(), v.end(), [](const auto &x, const auto &y) { return x.first > y.first; });
        std::vector<int32_t> flat;
        flat.reserve(2 * v.size());
        for (const auto &it : v) {
            flat.push_back(it.second.first);
            flat.push_back(it.second.second);
        }
        if (v.size() > (size_t)INT32_MAX / 2) return fail(JK_EINVAL, "too many persistent work items");
        jk_batch::Persist &q = b->persist[pr];
        if ((rc = b->alloc(&q.items, flat.size()))) return rc;
        HIPCHK(hipMemcpy(q.items, flat.data(), sizeof(int32_t) * flat.size(), hipMemcpyHostToDevice));
        q.nitems = (int)v.size();
        // workgroups: enough 64-lane waves to fill every CU several times
        q.grid = (int)std::min<int64_t>(q.nitems, (int64_t)std::max(ncu, 1) * 16);
    }
    if ((rc = b->alloc(&b->d_pctr, 2))) return rc;
    if (!b->hdesc.empty())
        HIPCHK(hipMemcpy(b->d_desc, b->hdesc.data(), sizeof(BatchDesc) * b->hdesc.size(), hipMemcpyHostToDevice));
    HIPCHK(hipHostMalloc((void **)&b->h_stage, sizeof(MolDesc) * nmol, hipHostMallocDefault));
    HIPCHK(hipEventCreateWithFlags(&b->stage_ev, hipEventDisableTiming));
    HIPCHK(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    // parallel branches of the graph (JK_BATCH_BRANCHES, default 4; all
    // streams at the default priority)
    {
        const char *nb = getenv("JK_BATCH_BRANCHES");
        const int v = nb && *nb ? atoi(nb) : 4;
        b->nbranch = std::max(1, std::min(v, (int)jk_batch::MAXBRANCH));
    }
    b->branch[0] = b->cap;
    for (int k = 1; k < b->nbranch; ++k) {
        HIPCHK(hipStreamCreateWithFlags(&b->branch[k], hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    *out = b.release();
    return JK_OK;
}

extern "C" int jk_batch_execute(jk_batch *b, const double *const *D, double *const *J, double *const *K, void *stream) {
    if (!b) return fail(JK_EINVAL, "batch is NULL");
    if (!D || !J || !K) return fail(JK_EINVAL, "D, J and K pointer arrays must be non-NULL");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev != b->device) return fail(JK_EINVAL, "batch was created on device %d, current device is %d", b->device, dev);
    // every pointer is checked before the cached table changes
    for (int m = 0; m < b->nmol; ++m)
        if (!D[m] || !J[m] || !K[m]) return fail(JK_EINVAL, "molecule %d: NULL D, J or K", m);
    hipStream_t s = (hipStream_t)stream;
    bool changed = false;
    for (int m = 0; m < b->nmol; ++m) {
        MolDesc &md = b->hmol[m];
        if (md.D != D[m] || md.J != J[m] || md.K != K[m]) {
            md.D = D[m];
            md.J = J[m];
            md.K = K[m];
            changed = true;
        }
    }
    if (changed) {
        // the previous upload from the staging buffer must have completed
        HIPCHK(hipEventSynchronize(b->stage_ev));
        std::memcpy(b->h_stage, b->hmol.data(), sizeof(MolDesc) * b->nmol);
        HIPCHK(hipMemcpyAsync(b->d_mol, b->h_stage, sizeof(MolDesc) * b->nmol, hipMemcpyHostToDevice, s));
        HIPCHK(hipEventRecord(b->stage_ev, s));
    }
    if (!b->exec) {
        HIPCHK(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        const int rc = record(b);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(b->cap, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        HIPCHK(e);
        b->graph = g;
        HIPCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(b->exec, s));
    return JK_OK;
}

extern "C" int jk_batch_stats(const jk_batch *b, int64_t *nquartets, int64_t *nquartets_fp32) {
    if (!b) return fail(JK_EINVAL, "batch is NULL");
    const size_t per = (size_t)NSEL_SLOTS * NSEL_STRIDE;
    std::vector<unsigned long long> raw(b->hdesc.size() * per);
    HIPCHK(hipDeviceSynchronize());
    if (!raw.empty())
        HIPCHK(hipMemcpy(raw.data(), b->d_ctr, sizeof(unsigned long long) * raw.size(), hipMemcpyDeviceToHost));
    int64_t n = 0, n32 = 0;
    for (size_t d = 0; d < b->hdesc.size(); ++d) {
        int64_t c = b->fixed[d];
        if (c < 0) {
            c = 0;
            for (int j = 0; j < NSEL_SLOTS; ++j) c += (int64_t)raw[d * per + (size_t)j * NSEL_STRIDE];
        }
        n += c;
        if (b->dprec[d] == 1) n32 += c;
    }
    if (nquartets) *nquartets = n;
    if (nquartets_fp32) *nquartets_fp32 = n32;
    return JK_OK;
}

extern "C" void jk_batch_destroy(jk_batch *b) { delete b; }
