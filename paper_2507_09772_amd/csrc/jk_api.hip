// jk_api.hip -- host planner and C ABI of the J/K library (include/jk.h),
// plus the small helper kernels: primitive-pair builder, Schwarz reduction,
// spherical <-> Cartesian transforms, density block maxima, finalisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/jk.h"
#include "jk_registry.h"
#include "tables/jk_tables.h"
#include "tables/jk_tables_mom.h"
#include "jk_internal.h"

#include <dlfcn.h>

namespace jk {
ClassEntry g_classes[NCLS];
}

using namespace jk;

// Tuning table: kernel family per (class, precision); 0 = built-in default.
// Loaded from the shipped per-device file at library load, settable through
// jk_tune_set, read by jk_plan_create.
static int32_t g_tune[NCLS][2];
// Row mode per (class, precision): 0 default (allowed), 1 allowed, 2 off.
static int32_t g_row[NCLS][2];
static void ensure_tuning();
static int launch_counts(const jk_plan *P, std::vector<int64_t> *out);

// Task shape per class (host side; 0 = default): bras with at least
// min_kets kets run in row mode (the default 192), and a row task covers at
// most chunk kets of one bra (by default row_chunk of the family; a set
// value applies to the row tasks of every family).
static const int ROW_MIN_KETS = 192;
static int32_t g_minkets[NCLS];
static int32_t g_chunk[NCLS];
// Mixed-precision split per class: 0 default (split), 1 split, 2 the whole
// class in double precision in mixed builds.
static int32_t g_split[NCLS];

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

extern "C" const char *jk_last_error(void) { return g_err.c_str(); }

// ---------------------------------------------------------------------------
// device tables (one copy per device, kept until the process ends)
// ---------------------------------------------------------------------------
static Tables g_tab[64];
static bool g_tab_ok[64];

template <typename T>
static int upload(T **dst, const T *src, size_t n) {
    HIPCHK(hipMalloc(dst, sizeof(T) * n));
    HIPCHK(hipMemcpy(*dst, src, sizeof(T) * n, hipMemcpyHostToDevice));
    return 0;
}

static int tables_for_device(Tables *out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(JK_EDEVICE, "device index %d out of range", dev);
    if (!g_tab_ok[dev]) {
        Tables t{};
        std::vector<float> f(JKT_RYS_NCOEF);
        for (int i = 0; i < JKT_RYS_NCOEF; ++i) f[i] = (float)jkt_rys_coef[i];
        int rc;
        if ((rc = upload((double **)&t.rys, jkt_rys_coef, JKT_RYS_NCOEF))) return rc;
        if ((rc = upload((float **)&t.rys32, f.data(), f.size()))) return rc;
        std::vector<float> hx(JKT_HERM_N), hw(JKT_HERM_N);
        for (int i = 0; i < JKT_HERM_N; ++i) { hx[i] = (float)jkt_herm_x2[i]; hw[i] = (float)jkt_herm_w[i]; }
        if ((rc = upload((double **)&t.hx2, jkt_herm_x2, JKT_HERM_N))) return rc;
        if ((rc = upload((double **)&t.hw, jkt_herm_w, JKT_HERM_N))) return rc;
        if ((rc = upload((float **)&t.hx2_32, hx.data(), hx.size()))) return rc;
        if ((rc = upload((float **)&t.hw32, hw.data(), hw.size()))) return rc;
        const size_t nb = sizeof(jkt_boys) / sizeof(double);
        std::vector<float> bf(nb);
        for (size_t i = 0; i < nb; ++i) bf[i] = (float)jkt_boys[i];
        if ((rc = upload((double **)&t.boys, jkt_boys, nb))) return rc;
        if ((rc = upload((float **)&t.boys32, bf.data(), nb))) return rc;
        if ((rc = upload((double **)&t.mom, jkt_mom, (size_t)JKT_MOM_NT * JKT_MOM_COLS))) return rc;
        g_tab[dev] = t;
        g_tab_ok[dev] = true;
    }
    *out = g_tab[dev];
    return 0;
}

// ---------------------------------------------------------------------------
// helper kernels
// ---------------------------------------------------------------------------

// One thread per shell pair: all primitive pairs of the pair.
__global__ void k_pair_build(ShellDev sh, PairRec *pairs, int npair, PrimPair *pp) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npair) return;
    const PairRec pr = pairs[t];
    const int I = pr.ish, J = pr.jsh;
    const double *A = sh.coords + 3 * sh.atom[I];
    const double *B = sh.coords + 3 * sh.atom[J];
    const double ab2 = (A[0] - B[0]) * (A[0] - B[0]) + (A[1] - B[1]) * (A[1] - B[1]) + (A[2] - B[2]) * (A[2] - B[2]);
    const int nj = sh.nprim[J];
    for (int ip = 0; ip < sh.nprim[I]; ++ip)
        for (int jp = 0; jp < nj; ++jp) {
            const double a = sh.exps[sh.poff[I] + ip], b = sh.exps[sh.poff[J] + jp];
            const double p = a + b;
            PrimPair r;
            r.p = p;
            r.h = 0.5 / p;
            r.kp = sh.coefs[sh.poff[I] + ip] * sh.coefs[sh.poff[J] + jp] * exp(-a * b / p * ab2) / p;
            r.pad = 0.0;
            for (int x = 0; x < 3; ++x) {
                r.P[x] = (a * A[x] + b * B[x]) / p;
                r.PA[x] = r.P[x] - A[x];
            }
            pp[pr.pp_off + (ip * nj + jp) * pr.pp_stride] = r;
        }
}

// q of each pair from its exported diagonal block (IJ|IJ): sqrt(max_ab |(ab|ab)|)
__global__ void k_schwarz(const double *blocks, int nab, const int32_t *pair_ids, int n, PairRec *pairs) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double *b = blocks + (int64_t)t * nab * nab;
    double m = 0.0;
    for (int e = 0; e < nab; ++e) m = fmax(m, fabs(b[e * nab + e]));
    pairs[pair_ids[t]].q = sqrt(m);
}

__global__ void k_fill_i32(int32_t *p, int n) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) p[t] = 0;
}

// The fixed-order limbs of elements 0..n-1 (limbs L apart) into doubles, in
// place over the first limb: the smallest part first, the same order for
// every element and every build.
__global__ void k_det_collapse(double *p, int64_t L, int64_t n) {
    const long long *q = reinterpret_cast<const long long *>(p);
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const long long q0 = q[t], q1 = q[t + L], q2 = q[t + 2 * L];
        p[t] = ((double)q2 * 0x1p-96 + (double)q1 * 0x1p-56) + (double)q0 * 0x1p-16;
    }
}

__global__ void k_jp_scatter(const PairRec *pairs, const int32_t *lsh, const double *jp, int64_t jpstride, double *Jc,
                             int64_t mstride, int naoc, int npair, int64_t nt) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x)
        jp_scatter_elem(pairs, lsh, jp, jpstride, Jc, mstride, naoc, npair, t);
}

__global__ void k_fill(double *p, int64_t n, double v) {
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) p[t] = v;
}


// Dc[s][a][b] = sum_{m, n} T_I[m][a] D[s][m][n] T_J[n][b]  (D spherical)
__global__ void k_sph_to_cart(AoMaps m, const double *D, double *Dc, int nao, int naoc, int nset) {
    const int64_t tot = (int64_t)nset * naoc * naoc;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x)
        Dc[t] = sph_to_cart_elem(m, D, nao, naoc, t);
}

// out[s] (+)= T (X + X^T) T^T, or X + X^T for Cartesian bases
__global__ void k_finalize(AoMaps m, const double *X, double *out, int nao, int naoc, int nset, int spherical, int accumulate) {
    const int64_t tot = (int64_t)nset * nao * nao;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const double v = finalize_elem(m, X, nao, naoc, spherical, t);
        out[t] = accumulate ? out[t] + v : v;
    }
}

// dmax[I][J] = max_s max_{a in I, b in J} |Dc[s][a][b]|
__global__ void k_dmax(const double *Dc, const int32_t *aoc, const int32_t *l, int ns, int naoc, int nset, double *dmax) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ns * ns) return;
    dmax[t] = dmax_elem(Dc, aoc, l, ns, naoc, nset, t);
}

// dmax[ns * ns] = the largest entry of the table (one workgroup).
__global__ void __launch_bounds__(256) k_dmax_all(double *dmax, int ns) {
    __shared__ double part[256];
    double m = 0.0;
    for (int t = threadIdx.x; t < ns * ns; t += 256) m = fmax(m, dmax[t]);
    part[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] = fmax(part[threadIdx.x], part[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dmax[ns * ns] = part[0];
}

template <int N, typename R>
__global__ void k_rys_eval(Tables tab, const double *T, int n, double *u, double *w) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    R uu[N], ww[N];
    rys_roots<N, R>(T[t], tab, uu, ww);
    for (int i = 0; i < N; ++i) {
        u[t * N + i] = (double)uu[i];
        w[t * N + i] = (double)ww[i];
    }
}

template <typename R>
__global__ void k_boys_eval(Tables tab, const double *T, int n, double *out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    R u, w;
    rys1<R>(T[t], TabSel<R>::boys(tab), u, w);
    out[2 * t] = (double)w;            // F_0
    out[2 * t + 1] = (double)(u * w);  // F_1
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------



static int validate_basis(const jk_basis *b) {
    if (!b) return fail(JK_EINVAL, "basis is NULL");
    if (b->nshell < 1 || b->natom < 1) return fail(JK_EINVAL, "nshell and natom must be >= 1");
    if (!b->l || !b->nprim || !b->atom || !b->exps || !b->coefs || !b->coords) return fail(JK_EINVAL, "NULL basis array");
    if (b->spherical != 0 && b->spherical != 1) return fail(JK_EINVAL, "spherical must be 0 or 1");
    int64_t np = 0;
    for (int i = 0; i < b->nshell; ++i) {
        if (b->l[i] < 0 || b->l[i] > JK_LMAX) return fail(JK_EINVAL, "shell %d: l=%d outside 0..%d", i, b->l[i], JK_LMAX);
        if (b->l[i] > LMAX_BUILT) return fail(JK_EUNSUPPORTED, "shell %d: l=%d above the built maximum %d", i, b->l[i], LMAX_BUILT);
        if (b->nprim[i] < 1 || b->nprim[i] > JK_MAXPRIM) return fail(JK_EINVAL, "shell %d: nprim=%d outside 1..%d", i, b->nprim[i], JK_MAXPRIM);
        if (b->atom[i] < 0 || b->atom[i] >= b->natom) return fail(JK_EINVAL, "shell %d: atom %d out of range", i, b->atom[i]);
        np += b->nprim[i];
    }
    for (int64_t k = 0; k < np; ++k) {
        if (!(std::isfinite(b->exps[k]) && b->exps[k] > 0.0)) return fail(JK_EINVAL, "primitive %lld: exponent must be finite and > 0", (long long)k);
        if (!std::isfinite(b->coefs[k])) return fail(JK_EINVAL, "primitive %lld: coefficient not finite", (long long)k);
    }
    for (int k = 0; k < 3 * b->natom; ++k)
        if (!std::isfinite(b->coords[k])) return fail(JK_EINVAL, "coordinate %d not finite", k);
    return 0;
}

// per primitive quartet algorithmic FLOPs (roots, recurrences, assembly) and
// per contracted quartet digestion FLOPs (J and K, one density)
static double flops_prim(int li, int lj, int lk, int ll) {
    const int nr = nroots(li, lj, lk, ll);
    const double nc = (double)ncart(li) * ncart(lj) * ncart(lk) * ncart(ll);
    const double rec = 5.0 * (li + lj + 1) * (lk + ll + 1) + 2.0 * (li + 1) * (lj + 1) * (lk + ll + 1) +
                       2.0 * (li + 1) * (lj + 1) * (lk + 1) * (ll + 1);
    const double roots = nr == 1 ? 40.0 : 56.0 * nr;
    return 3.0 * nr * nc + 3.0 * nr * rec + roots + 30.0;
}
static double flops_digest(int li, int lj, int lk, int ll) {
    return 12.0 * ncart(li) * ncart(lj) * ncart(lk) * ncart(ll);
}

static int launch_export(jk_plan *P, int li, int lj, int lk, int ll, int precision, const int32_t *d_qb, const int32_t *d_qk,
                         int nq, double *d_out, hipStream_t s) {
    const ClassEntry &e = g_classes[class_id(li, lj, lk, ll)];
    Launcher f = precision == JK_FP64 ? e.ex64 : e.ex32;
    if (!f) return fail(JK_EUNSUPPORTED, "class (%d%d|%d%d) not built", li, lj, lk, ll);
    JkArgs a{};
    a.pairs = P->d_pairs;
    a.pp = P->d_pp;
    a.q_bra = d_qb;
    a.q_ket = d_qk;
    a.nq = nq;
    a.out = d_out;
    a.tab = P->tab;
    HIPCHK(f(a, s));
    return 0;
}

extern "C" int jk_plan_create(const jk_basis *basis, double cutoff, jk_plan **out) {
    if (!out) return fail(JK_EINVAL, "out is NULL");
    ensure_tuning();
    *out = nullptr;
    int rc = validate_basis(basis);
    if (rc) return rc;
    if (!(std::isfinite(cutoff) && cutoff >= 0.0)) return fail(JK_EINVAL, "cutoff must be finite and >= 0");
    const auto t0 = std::chrono::steady_clock::now();
    jk_plan *P = new (std::nothrow) jk_plan();
    if (!P) return fail(JK_ENOMEM, "host allocation failed");
    std::unique_ptr<jk_plan> guard(P);
    HIPCHK(hipGetDevice(&P->device));
    if ((rc = tables_for_device(&P->tab))) return rc;
    {
        const char *ns = getenv("JK_STREAMS");
        const int nsv = ns && *ns ? atoi(ns) : 4;
        P->nstream = std::max(1, std::min(nsv, (int)jk_plan::MAXSTREAM));
    }
    HIPCHK(hipEventCreateWithFlags(&P->fork_ev, hipEventDisableTiming));
    for (int k = 1; k < P->nstream; ++k) {
        HIPCHK(hipStreamCreateWithFlags(&P->streams[k], hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&P->join_ev[k], hipEventDisableTiming));
    }
    {
        const char *nr = getenv("JK_NO_ROW");
        P->no_row = nr && nr[0] == '1';
        const char *nd = getenv("JK_NO_DSTAGE");
        P->no_dstage = nd && nd[0] == '1';
    }
    const int ns = P->ns = basis->nshell;
    P->natom = basis->natom;
    P->sph = basis->spherical;
    P->cutoff = cutoff;
    P->l.assign(basis->l, basis->l + ns);
    P->nprim.assign(basis->nprim, basis->nprim + ns);
    P->atom.assign(basis->atom, basis->atom + ns);
    P->poff.resize(ns + 1);
    P->aoc.resize(ns + 1);
    P->aoe.resize(ns + 1);
    P->poff[0] = P->aoc[0] = P->aoe[0] = 0;
    for (int i = 0; i < ns; ++i) {
        P->poff[i + 1] = P->poff[i] + P->nprim[i];
        P->aoc[i + 1] = P->aoc[i] + ncart(P->l[i]);
        P->aoe[i + 1] = P->aoe[i] + (P->sph ? 2 * P->l[i] + 1 : ncart(P->l[i]));
    }
    P->naoc = P->aoc[ns];
    P->nao = P->aoe[ns];
    const int nprim_tot = P->poff[ns];

    // shell types (l, nprim), ordered by l then nprim, both descending
    std::vector<std::pair<int, int>> keys;
    for (int i = 0; i < ns; ++i) keys.push_back({P->l[i], P->nprim[i]});
    std::sort(keys.begin(), keys.end(), [](auto &x, auto &y) { return x > y; });
    keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
    const int ntype = (int)keys.size();
    std::vector<int> stype(ns);
    for (int i = 0; i < ns; ++i)
        stype[i] = (int)(std::find(keys.begin(), keys.end(), std::make_pair(P->l[i], P->nprim[i])) - keys.begin());

    // oriented pairs, grouped by pair type (t1 <= t2)
    std::vector<std::vector<PairRec>> by_type(ntype * ntype);
    for (int I = 0; I < ns; ++I)
        for (int J = 0; J <= I; ++J) {
            int a = I, b = J;
            if (stype[a] > stype[b]) std::swap(a, b);
            PairRec r{};
            r.ish = a;
            r.jsh = b;
            r.aoi = P->aoc[a];
            r.aoj = P->aoc[b];
            r.npp = P->nprim[a] * P->nprim[b];
            const double *A = basis->coords + 3 * P->atom[a], *B = basis->coords + 3 * P->atom[b];
            for (int x = 0; x < 3; ++x) r.ab[x] = A[x] - B[x];
            by_type[stype[a] * ntype + stype[b]].push_back(r);
        }
    // Primitive pairs are stored type-major: the k-th primitive pair of the
    // i-th pair of a type sits at base(type) + k * count(type) + i, so a wave
    // reading consecutive pairs of one type reads consecutive records.
    std::vector<int> ptype_first, ptype_count, ptype_key, ptype_ppbase;  // pair types present
    int64_t npp_tot = 0;
    for (int t = 0; t < ntype * ntype; ++t) {
        if (by_type[t].empty()) continue;
        ptype_first.push_back((int)P->hpairs.size());
        ptype_count.push_back((int)by_type[t].size());
        ptype_key.push_back(t);
        ptype_ppbase.push_back((int)npp_tot);
        for (auto &r : by_type[t]) P->hpairs.push_back(r);
        npp_tot += (int64_t)by_type[t].size() * by_type[t][0].npp;
    }
    if (npp_tot > INT32_MAX) return fail(JK_EUNSUPPORTED, "too many primitive pairs");
    const int npair = (int)P->hpairs.size();
    const int npt0 = (int)ptype_first.size();
    // the pair-ordered J' buffer has the same type-major layout
    std::vector<int64_t> ptype_jpbase(npt0);
    int64_t jp_tot = 0;
    for (int pt = 0; pt < npt0; ++pt) {
        const PairRec &r0 = P->hpairs[ptype_first[pt]];
        ptype_jpbase[pt] = jp_tot;
        jp_tot += (int64_t)ptype_count[pt] * ncart(P->l[r0.ish]) * ncart(P->l[r0.jsh]);
    }
    if (jp_tot > INT32_MAX) return fail(JK_EUNSUPPORTED, "too many shell-pair elements");
    P->njp = jp_tot;
    auto place_pairs = [&]() {
        for (int pt = 0; pt < npt0; ++pt)
            for (int k = 0; k < ptype_count[pt]; ++k) {
                PairRec &r = P->hpairs[ptype_first[pt] + k];
                r.pp_off = ptype_ppbase[pt] + k;
                r.pp_stride = ptype_count[pt];
                r.jp_off = (int32_t)(ptype_jpbase[pt] + k);
            }
        P->pair_of.assign((size_t)ns * ns, -1);
        for (int p = 0; p < npair; ++p) {
            P->pair_of[(size_t)P->hpairs[p].ish * ns + P->hpairs[p].jsh] = p;
            P->pair_of[(size_t)P->hpairs[p].jsh * ns + P->hpairs[p].ish] = p;
        }
    };
    place_pairs();

    // device copies of the basis and the pair data
    int32_t *d_l, *d_np, *d_poff, *d_atom, *d_aoc, *d_aoe;
    double *d_exps, *d_coefs, *d_coords;
    if ((rc = P->put(&d_l, P->l)) || (rc = P->put(&d_np, P->nprim)) || (rc = P->put(&d_poff, P->poff)) ||
        (rc = P->put(&d_atom, P->atom)) || (rc = P->put(&d_aoc, P->aoc)) || (rc = P->put(&d_aoe, P->aoe)))
        return rc;
    if ((rc = P->put(&d_exps, std::vector<double>(basis->exps, basis->exps + nprim_tot))) ||
        (rc = P->put(&d_coefs, std::vector<double>(basis->coefs, basis->coefs + nprim_tot))) ||
        (rc = P->put(&d_coords, std::vector<double>(basis->coords, basis->coords + 3 * P->natom))))
        return rc;
    P->sh = ShellDev{d_l, d_np, d_poff, d_atom, d_exps, d_coefs, d_coords};
    if ((rc = P->put(&P->d_pairs, P->hpairs))) return rc;
    if ((rc = P->alloc(&P->d_pp, npp_tot))) return rc;
    hipLaunchKernelGGL(k_pair_build, dim3((npair + 127) / 128), dim3(128), 0, 0, P->sh, P->d_pairs, npair, P->d_pp);
    HIPCHK(hipGetLastError());

    // Schwarz factors: exported diagonal blocks (IJ|IJ) per pair type
    for (size_t pt = 0; pt < ptype_first.size(); ++pt) {
        const int first = ptype_first[pt], cnt = ptype_count[pt];
        const PairRec &r0 = P->hpairs[first];
        const int li = P->l[r0.ish], lj = P->l[r0.jsh];
        const int nab = ncart(li) * ncart(lj);
        std::vector<int32_t> ids(cnt);
        std::iota(ids.begin(), ids.end(), first);
        int32_t *d_ids;
        double *d_blk;
        if ((rc = P->put(&d_ids, ids))) return rc;
        if ((rc = P->alloc(&d_blk, (size_t)cnt * nab * nab))) return rc;
        if ((rc = launch_export(P, li, lj, li, lj, JK_FP64, d_ids, d_ids, cnt, d_blk, 0))) return rc;
        hipLaunchKernelGGL(k_schwarz, dim3((cnt + 127) / 128), dim3(128), 0, 0, d_blk, nab, d_ids, cnt, P->d_pairs);
        HIPCHK(hipGetLastError());
        HIPCHK(hipDeviceSynchronize());
        HIPCHK(hipFree(d_blk));
        P->allocs.erase(std::find(P->allocs.begin(), P->allocs.end(), (void *)d_blk));
    }
    HIPCHK(hipMemcpy(P->hpairs.data(), P->d_pairs, sizeof(PairRec) * npair, hipMemcpyDeviceToHost));
    // renumber the pairs of each type by q descending (ties keep their order),
    // so each type's screening list is a contiguous id range, then rebuild
    // the primitive pairs in that order
    for (int pt = 0; pt < npt0; ++pt)
        std::stable_sort(P->hpairs.begin() + ptype_first[pt], P->hpairs.begin() + ptype_first[pt] + ptype_count[pt],
                         [](const PairRec &x, const PairRec &y) { return x.q > y.q; });
    place_pairs();
    HIPCHK(hipMemcpy(P->d_pairs, P->hpairs.data(), sizeof(PairRec) * npair, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_pair_build, dim3((npair + 127) / 128), dim3(128), 0, 0, P->sh, P->d_pairs, npair, P->d_pp);
    HIPCHK(hipGetLastError());
    P->Qsh.assign((size_t)ns * ns, 0.0);
    double qmax = 0.0;
    for (auto &r : P->hpairs) {
        P->Qsh[(size_t)r.ish * ns + r.jsh] = P->Qsh[(size_t)r.jsh * ns + r.ish] = r.q;
        qmax = std::max(qmax, r.q);
    }

    // per pair type: pairs that can pass the test with some partner, by q descending
    const int npt = (int)ptype_first.size();
    std::vector<std::vector<int32_t>> sorted(npt);
    std::vector<std::vector<double>> sortedq(npt);
    std::vector<int32_t *> d_sorted(npt, nullptr);
    for (int pt = 0; pt < npt; ++pt) {
        auto &v = sorted[pt];
        for (int k = 0; k < ptype_count[pt]; ++k) {
            const int p = ptype_first[pt] + k;
            if (P->hpairs[p].q * qmax >= cutoff && P->hpairs[p].q > 0.0) v.push_back(p);
        }
        std::stable_sort(v.begin(), v.end(), [&](int x, int y) { return P->hpairs[x].q > P->hpairs[y].q; });
        for (int p : v) sortedq[pt].push_back(P->hpairs[p].q);
        if (!v.empty() && (rc = P->put(&d_sorted[pt], v))) return rc;
    }
    // shells of each type (the compressed column segments of row mode)
    std::vector<std::vector<int32_t>> tsh(ntype);
    std::vector<int32_t> tpos(ns);
    for (int i = 0; i < ns; ++i) {
        tpos[i] = (int32_t)tsh[stype[i]].size();
        tsh[stype[i]].push_back(i);
    }
    std::vector<int32_t *> d_tsh(ntype, nullptr);
    for (int t = 0; t < ntype; ++t)
        if ((rc = P->put(&d_tsh[t], tsh[t]))) return rc;
    if ((rc = P->put(&P->d_tpos, tpos))) return rc;
    // classes: unordered pairs of pair types, bra = larger (l1, l2), ties by type index
    auto lkey = [&](int pt) { const PairRec &r = P->hpairs[ptype_first[pt]]; return std::make_pair(P->l[r.ish], P->l[r.jsh]); };
    int64_t nq_tot = 0, npq_tot = 0;
    double flops_tot = 0.0;
    for (int x = 0; x < npt; ++x)
        for (int y = 0; y <= x; ++y) {
            int bt = x, kt = y;
            if (lkey(kt) > lkey(bt)) std::swap(bt, kt);
            if (sorted[bt].empty() || sorted[kt].empty()) continue;
            ClassTask c{};
            c.li = lkey(bt).first; c.lj = lkey(bt).second; c.lk = lkey(kt).first; c.ll = lkey(kt).second;
            c.bt = bt; c.kt = kt; c.same = bt == kt;
            c.npb = P->hpairs[ptype_first[bt]].npp;
            c.npk = P->hpairs[ptype_first[kt]].npp;
            const ClassEntry &ce = g_classes[class_id(c.li, c.lj, c.lk, c.ll)];
            const bool avail[3] = {ce.tiles[0][0] != nullptr, ce.tiles[1][0] != nullptr, ce.row[2][0] != nullptr};
            if (!avail[0] && !avail[1]) return fail(JK_EUNSUPPORTED, "class (%d%d|%d%d) not built", c.li, c.lj, c.lk, c.ll);
            for (int pr = 0; pr < 2; ++pr) {
                int f = g_tune[class_id(c.li, c.lj, c.lk, c.ll)][pr];
                if (f < 1 || f > 3 || !avail[f - 1]) f = default_family(c.li, c.lj, c.lk, c.ll);
                if (!avail[f - 1]) f = 3 - f;
                c.fam[pr] = f;
                c.row_ok[pr] = g_row[class_id(c.li, c.lj, c.lk, c.ll)][pr] != 2;
                c.split = g_split[class_id(c.li, c.lj, c.lk, c.ll)] != 2;
                c.row_short[pr] = g_row[class_id(c.li, c.lj, c.lk, c.ll)][pr] == 3;
            }
            std::vector<int32_t> bl, cn, to[2];
            const auto &kq = sortedq[kt];
            int64_t tiles[2] = {0, 0};
            for (size_t i = 0; i < sorted[bt].size(); ++i) {
                const double qb = sortedq[bt][i];
                // kets j with qb * kq[j] >= cutoff form a prefix
                size_t lo = 0, hi = kq.size();
                while (lo < hi) {
                    const size_t mid = (lo + hi) / 2;
                    if (qb * kq[mid] >= cutoff) lo = mid + 1;
                    else hi = mid;
                }
                size_t cnt = lo;
                if (c.same) cnt = std::min(cnt, i + 1);
                if (cnt == 0) continue;
                bl.push_back(sorted[bt][i]);
                cn.push_back((int32_t)cnt);
                for (int f = 0; f < 2; ++f) {
                    to[f].push_back((int32_t)tiles[f]);
                    const int qpt = quartets_per_tile(f + 1, c.li, c.lj, c.lk, c.ll);
                    tiles[f] += (cnt + qpt - 1) / qpt;
                }
                c.nq += cnt;
            }
            if (c.nq == 0) continue;
            if (tiles[0] > INT32_MAX || tiles[1] > INT32_MAX || c.nq > INT32_MAX)
                return fail(JK_EUNSUPPORTED, "class (%d%d|%d%d) has too many quartets", c.li, c.lj, c.lk, c.ll);
            c.nbra = (int)bl.size();
            c.npq = c.nq * c.npb * c.npk;
            c.flops = (double)c.npq * flops_prim(c.li, c.lj, c.lk, c.ll) + (double)c.nq * flops_digest(c.li, c.lj, c.lk, c.ll);
            if ((rc = P->put(&c.d_bra, bl)) || (rc = P->put(&c.d_cnt, cn))) return rc;
            for (int f = 0; f < 2; ++f) {
                c.ntiles[f] = (int)tiles[f];
                if (avail[f] && (rc = P->put(&c.d_tile[f], to[f]))) return rc;
            }
            c.d_ket = d_sorted[kt];
            // row mode split: bras with a long ket prefix get a workgroup each
            {
                const int tK = ptype_key[kt] / ntype, tL = ptype_key[kt] % ntype;
                c.ncolK = (int)tsh[tK].size() * ncart(c.lk);
                c.ncolL = (int)tsh[tL].size() * ncart(c.ll);
                c.seg_same = tK == tL;
                c.d_tshK = d_tsh[tK];
                c.d_tshL = d_tsh[tL];
                std::vector<int32_t> rows, sb, scn, sto[2];
                int64_t st[2] = {0, 0};
                for (size_t i = 0; i < bl.size(); ++i) {
                    const int minkets = g_minkets[class_id(c.li, c.lj, c.lk, c.ll)] > 0
                                            ? g_minkets[class_id(c.li, c.lj, c.lk, c.ll)] : ROW_MIN_KETS;
                    if (cn[i] >= minkets) {
                        rows.push_back((int32_t)i);
                        c.nq_row += cn[i];
                        continue;
                    }
                    // short bra: one 64-lane row task over all its kets
                    c.h_srowt.push_back((int32_t)i);
                    c.h_srowt.push_back(0);
                    c.h_srowt.push_back(cn[i]);
                    sb.push_back(bl[i]);
                    scn.push_back(cn[i]);
                    for (int f = 0; f < 2; ++f) {
                        sto[f].push_back((int32_t)st[f]);
                        const int qpt = quartets_per_tile(f + 1, c.li, c.lj, c.lk, c.ll);
                        st[f] += (cn[i] + qpt - 1) / qpt;
                    }
                }
                c.nrow = (int)rows.size();
                c.nsbra = (int)sb.size();
                if (c.nrow > 0 && (ce.row[0][0] || ce.row[1][0] || ce.row[2][0])) {
                    // row tasks: (list position, first ket, end ket), each long
                    // bra cut into near-equal chunks of at most row_chunk kets
                    for (int f = 0; f < 3; ++f) {
                        if (!ce.row[f][0]) continue;
                        const int gch = g_chunk[class_id(c.li, c.lj, c.lk, c.ll)];
                        const int ch = gch > 0 ? gch : row_chunk(f + 1, c.li, c.lj, c.lk, c.ll);
                        std::vector<int32_t> tasks;
                        for (int32_t i : rows) {
                            const int64_t n = cn[i], nch = (n + ch - 1) / ch, len = (n + nch - 1) / nch;
                            for (int64_t j = 0; j < n; j += len) {
                                tasks.push_back(i);
                                tasks.push_back((int32_t)j);
                                tasks.push_back((int32_t)std::min<int64_t>(n, j + len));
                            }
                        }
                        c.nrowc[f] = (int)(tasks.size() / 3);
                        if ((rc = P->put(&c.d_rowc[f], tasks))) return rc;
                        c.h_rowc[f] = tasks;
                    }
                    if (c.nsbra > 0) {
                        if ((rc = P->put(&c.d_sbra, sb)) || (rc = P->put(&c.d_scnt, scn))) return rc;
                        for (int f = 0; f < 2; ++f) {
                            c.nstiles[f] = (int)st[f];
                            if (avail[f] && (rc = P->put(&c.d_stile[f], sto[f]))) return rc;
                        }
                    }
                } else {
                    c.nrow = 0;
                    c.nq_row = 0;
                }
                c.nsrow = (int)(c.h_srowt.size() / 3);
                if (c.nsrow > 0 && (ce.srow[0][0] || ce.srow[1][0] || ce.srow[2][0]) && (rc = P->put(&c.d_srowt, c.h_srowt)))
                    return rc;
            }
            nq_tot += c.nq;
            npq_tot += c.npq;
            flops_tot += c.flops;
            P->cls.push_back(c);
        }
    // heaviest classes first
    std::stable_sort(P->cls.begin(), P->cls.end(), [](const ClassTask &a, const ClassTask &b) { return a.flops > b.flops; });

    // AO maps for the spherical transforms
    std::vector<int32_t> shc(P->naoc), cc(P->naoc), she(P->nao), ce(P->nao);
    for (int i = 0; i < ns; ++i) {
        for (int k = 0; k < P->aoc[i + 1] - P->aoc[i]; ++k) { shc[P->aoc[i] + k] = i; cc[P->aoc[i] + k] = k; }
        for (int k = 0; k < P->aoe[i + 1] - P->aoe[i]; ++k) { she[P->aoe[i] + k] = i; ce[P->aoe[i] + k] = k; }
    }
    int32_t *d_shc, *d_cc, *d_she, *d_ce;
    double *d_c2s;
    if ((rc = P->put(&d_shc, shc)) || (rc = P->put(&d_cc, cc)) || (rc = P->put(&d_she, she)) || (rc = P->put(&d_ce, ce)) ||
        (rc = P->put(&d_c2s, std::vector<double>(jkt_c2s, jkt_c2s + JKT_C2S_N))))
        return rc;
    P->maps = AoMaps{d_shc, d_cc, d_she, d_ce, d_l, d_aoc, d_aoe, d_c2s};
    HIPCHK(hipDeviceSynchronize());

    P->stats.nquartets = nq_tot;
    P->stats.nprim_quartets = npq_tot;
    P->stats.nclasses = (int32_t)P->cls.size();
    P->stats.npairs = 0;
    for (auto &v : sorted) P->stats.npairs += (int32_t)v.size();
    P->stats.model_flops = flops_tot;
    P->stats.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = guard.release();
    return JK_OK;
}

extern "C" void jk_plan_destroy(jk_plan *plan) { delete plan; }

extern "C" int jk_plan_info(const jk_plan *P, int32_t *nao, int32_t *nao_cart) {
    if (!P) return fail(JK_EINVAL, "plan is NULL");
    if (nao) *nao = P->nao;
    if (nao_cart) *nao_cart = P->naoc;
    return 0;
}

extern "C" int jk_plan_stats(const jk_plan *P, jk_stats *st) {
    if (!P || !st) return fail(JK_EINVAL, "NULL argument");
    *st = P->stats;
    st->nquartets_fp32 = 0;
    st->nquartets_evaluated = 0;
    if (P->last_nsel && !P->cls.empty()) {
        // the counters of the last build: [class][precision][kind]
        std::vector<int64_t> cnt;
        HIPCHK(hipDeviceSynchronize());
        const int rc = launch_counts(P, &cnt);
        if (rc) return rc;
        for (size_t k = 0; k < cnt.size(); ++k) {
            st->nquartets_evaluated += cnt[k];
            if ((k / 4) % 2 == 1) st->nquartets_fp32 += cnt[k];
        }
    }
    return 0;
}

// ---------------------------------------------------------------------------
// tuning table
// ---------------------------------------------------------------------------
static bool valid_class(int li, int lj, int lk, int ll) {
    return li >= lj && lk >= ll && li <= LMAX_BUILT && lk <= LMAX_BUILT && lj >= 0 && ll >= 0 &&
           (lk < li || (lk == li && ll <= lj));
}

static int tune_set_impl(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t precision, int32_t family) {
    if (!valid_class(li, lj, lk, ll)) return fail(JK_EINVAL, "(%d%d|%d%d) is not a canonical built class", li, lj, lk, ll);
    if (precision != JK_FP64 && precision != JK_FP32) return fail(JK_EINVAL, "precision must be JK_FP64 or JK_FP32");
    if (family < 0 || family > 3) return fail(JK_EINVAL, "family must be 0, 1, 2 or 3");
    const ClassEntry &e = g_classes[class_id(li, lj, lk, ll)];
    const bool built = family == 3 ? e.row[2][0] != nullptr : family ? e.tiles[family - 1][0] != nullptr : true;
    if (!built) return fail(JK_EUNSUPPORTED, "family %d is not built for (%d%d|%d%d)", family, li, lj, lk, ll);
    g_tune[class_id(li, lj, lk, ll)][precision == JK_FP32 ? 1 : 0] = family;
    return 0;
}

static int tune_set_row_impl(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t precision, int32_t row) {
    if (!valid_class(li, lj, lk, ll)) return fail(JK_EINVAL, "(%d%d|%d%d) is not a canonical built class", li, lj, lk, ll);
    if (precision != JK_FP64 && precision != JK_FP32) return fail(JK_EINVAL, "precision must be JK_FP64 or JK_FP32");
    if (row < 0 || row > 3)
        return fail(JK_EINVAL, "row must be 0 (default), 1 (long bras), 2 (off) or 3 (long and short bras)");
    g_row[class_id(li, lj, lk, ll)][precision == JK_FP32 ? 1 : 0] = row;
    return 0;
}

extern "C" int jk_tune_set(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t precision, int32_t family) {
    ensure_tuning();
    return tune_set_impl(li, lj, lk, ll, precision, family);
}

extern "C" int jk_tune_set_row(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t precision, int32_t row) {
    ensure_tuning();
    return tune_set_row_impl(li, lj, lk, ll, precision, row);
}

static int tune_set_shape_impl(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t min_kets, int32_t chunk) {
    if (!valid_class(li, lj, lk, ll)) return fail(JK_EINVAL, "(%d%d|%d%d) is not a canonical built class", li, lj, lk, ll);
    if (min_kets < 0 || min_kets > (1 << 24) || chunk < 0 || chunk > (1 << 24))
        return fail(JK_EINVAL, "min_kets and chunk must be in 0..2^24 (0: default)");
    g_minkets[class_id(li, lj, lk, ll)] = min_kets;
    g_chunk[class_id(li, lj, lk, ll)] = chunk;
    return 0;
}

extern "C" int jk_tune_set_shape(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t min_kets, int32_t chunk) {
    ensure_tuning();
    return tune_set_shape_impl(li, lj, lk, ll, min_kets, chunk);
}

static int tune_set_split_impl(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t split) {
    if (!valid_class(li, lj, lk, ll)) return fail(JK_EINVAL, "(%d%d|%d%d) is not a canonical built class", li, lj, lk, ll);
    if (split != 0 && split != 1) return fail(JK_EINVAL, "split must be 0 or 1");
    g_split[class_id(li, lj, lk, ll)] = split ? 1 : 2;
    return 0;
}

extern "C" int jk_tune_set_split(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t split) {
    ensure_tuning();
    return tune_set_split_impl(li, lj, lk, ll, split);
}

extern "C" int jk_tune_get(int32_t li, int32_t lj, int32_t lk, int32_t ll, int32_t precision, int32_t *family,
                           int32_t *available) {
    ensure_tuning();
    if (!valid_class(li, lj, lk, ll)) return fail(JK_EINVAL, "(%d%d|%d%d) is not a canonical built class", li, lj, lk, ll);
    if (precision != JK_FP64 && precision != JK_FP32) return fail(JK_EINVAL, "precision must be JK_FP64 or JK_FP32");
    const ClassEntry &e = g_classes[class_id(li, lj, lk, ll)];
    const int f = g_tune[class_id(li, lj, lk, ll)][precision == JK_FP32 ? 1 : 0];
    if (family) *family = f ? f : default_family(li, lj, lk, ll);
    if (available) *available = (e.tiles[0][0] ? 1 : 0) | (e.tiles[1][0] ? 2 : 0) | (e.row[2][0] ? 4 : 0);
    return 0;
}

static int tune_load_impl(const char *path) {
    if (!path) return fail(JK_EINVAL, "path is NULL");
    FILE *f = fopen(path, "r");
    if (!f) return fail(JK_EINVAL, "cannot open %s", path);
    char line[256];
    int n = 0, lineno = 0;
    while (fgets(line, sizeof line, f)) {
        ++lineno;
        if (line[0] == '#' || line[0] == '\n') continue;
        int li, lj, lk, ll, pr, fam, row = 0;
        if (strncmp(line, "split", 5) == 0) {
            int sp = 1;
            if (sscanf(line + 5, "%d %d %d %d %d", &li, &lj, &lk, &ll, &sp) != 5) {
                fclose(f);
                return fail(JK_EINVAL, "%s:%d: expected 'split li lj lk ll s'", path, lineno);
            }
            const int rc = tune_set_split_impl(li, lj, lk, ll, sp);
            if (rc) { fclose(f); return rc; }
            ++n;
            continue;
        }
        if (strncmp(line, "shape", 5) == 0) {
            int mk = 0, ch = 0;
            if (sscanf(line + 5, "%d %d %d %d %d %d", &li, &lj, &lk, &ll, &mk, &ch) != 6) {
                fclose(f);
                return fail(JK_EINVAL, "%s:%d: expected 'shape li lj lk ll min_kets chunk'", path, lineno);
            }
            const int rc = tune_set_shape_impl(li, lj, lk, ll, mk, ch);
            if (rc) { fclose(f); return rc; }
            ++n;
            continue;
        }
        const int got = sscanf(line, "%d %d %d %d %d %d %d", &li, &lj, &lk, &ll, &pr, &fam, &row);
        if (got != 6 && got != 7) {
            fclose(f);
            return fail(JK_EINVAL, "%s:%d: expected 'li lj lk ll precision family [row]'", path, lineno);
        }
        int rc = tune_set_impl(li, lj, lk, ll, pr, fam);
        if (!rc) rc = tune_set_row_impl(li, lj, lk, ll, pr, row);
        if (rc) { fclose(f); return rc; }
        ++n;
    }
    fclose(f);
    return 0;
}

// The shipped table for this device sits next to the library.  It is read
// once, on the first plan creation or tuning call: the kernel units register
// their classes from static initialisers, which must have run before the
// table's entries can be checked against the built families.
static std::once_flag g_tune_once;

static void load_default_tuning() {
    const char *env = getenv("JK_TUNE_DB");
    std::string path;
    if (env && *env) {
        path = env;
    } else {
        Dl_info info;
        if (!dladdr((void *)&load_default_tuning, &info) || !info.dli_fname) return;
        path = info.dli_fname;
        const size_t sl = path.rfind('/');
        path = (sl == std::string::npos ? std::string(".") : path.substr(0, sl)) + "/tune_gfx950.txt";
    }
    FILE *f = fopen(path.c_str(), "r");
    if (!f) return;
    fclose(f);
    const std::string keep = g_err;
    if (tune_load_impl(path.c_str()) != 0) fprintf(stderr, "libjk: tuning table %s ignored: %s\n", path.c_str(), g_err.c_str());
    g_err = keep;
}

static void ensure_tuning() { std::call_once(g_tune_once, load_default_tuning); }

extern "C" int jk_tune_load(const char *path) {
    ensure_tuning();
    return tune_load_impl(path);
}

extern "C" int jk_plan_schwarz(const jk_plan *P, double *Q) {
    if (!P || !Q) return fail(JK_EINVAL, "NULL argument");
    std::memcpy(Q, P->Qsh.data(), sizeof(double) * P->Qsh.size());
    return 0;
}

static int grid_for(int64_t n, int block) { return (int)std::min<int64_t>((n + block - 1) / block, 65536); }

static void drop_alloc(jk_plan *P, void *p) {
    if (!p) return;
    (void)hipFree(p);
    P->allocs.erase(std::find(P->allocs.begin(), P->allocs.end(), p));
}

// The plan's own scratch, grown on demand (jk_execute).
static int ensure_scratch(jk_plan *P, int nset, Scratch *sc, bool det = false) {
    const size_t m = (size_t)P->naoc * P->naoc;
    int rc;
    // the fixed-order limbs: one length for the three buffers, so that a
    // kernel finds every limb at the same distance
    const int64_t L = (int64_t)std::max(m * nset, (size_t)P->njp * nset);
    if (det && P->det_len < L) {
        drop_alloc(P, P->d_det);
        P->d_det = nullptr;
        P->det_len = 0;
        if ((rc = P->alloc(&P->d_det, 9 * (size_t)L))) return rc;
        P->det_len = L;
    }
    if (P->scratch_nset < nset) {
        drop_alloc(P, P->d_Jc);
        drop_alloc(P, P->d_Kc);
        drop_alloc(P, P->d_jp);
        P->d_Jc = P->d_Kc = P->d_jp = nullptr;
        P->scratch_nset = 0;
        if ((rc = P->alloc(&P->d_Jc, m * nset)) || (rc = P->alloc(&P->d_Kc, m * nset)) ||
            (rc = P->alloc(&P->d_jp, (size_t)P->njp * nset)))
            return rc;
        P->scratch_nset = nset;
    }
    if (P->sph && P->dc_nset < nset) {
        drop_alloc(P, P->d_Dc);
        P->d_Dc = nullptr;
        P->dc_nset = 0;
        if ((rc = P->alloc(&P->d_Dc, m * nset))) return rc;
        P->dc_nset = nset;
    }
    if (!P->d_dmax && (rc = P->alloc(&P->d_dmax, scratch_sizes(P, 1).dmax))) return rc;
    if (!P->d_nsel && (rc = P->alloc(&P->d_nsel, scratch_sizes(P, 1).nsel))) return rc;
    *sc = Scratch{P->d_Jc, P->d_Kc, P->d_Dc, P->d_jp, P->d_dmax, P->d_nsel};
    if (det) {
        sc->det = P->d_det;
        sc->detL = L;
    }
    return 0;
}

// Quartets each launch of the last build evaluated, [class][precision][kind]
// (device counters summed over their slots, or the host's count).
static int launch_counts(const jk_plan *P, std::vector<int64_t> *out) {
    const size_t nl = P->cls.size() * 8, per = (size_t)NSEL_SLOTS * NSEL_STRIDE;
    std::vector<unsigned long long> raw(nl * per);
    HIPCHK(hipMemcpy(raw.data(), P->last_nsel, sizeof(unsigned long long) * raw.size(), hipMemcpyDeviceToHost));
    out->assign(nl, 0);
    for (size_t k = 0; k < nl; ++k) {
        if (k < P->last_fixed.size() && P->last_fixed[k] >= 0) {
            (*out)[k] = P->last_fixed[k];
            continue;
        }
        int64_t s = 0;
        for (int j = 0; j < NSEL_SLOTS; ++j) s += (int64_t)raw[k * per + (size_t)j * NSEL_STRIDE];
        (*out)[k] = s;
    }
    return 0;
}

__global__ void k_fill_u64(unsigned long long *p, int n) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) p[t] = 0ull;
}

int check_execute_args(const jk_plan *P, const double *D, int32_t nset, int32_t flags, int32_t precision,
                              double mix_threshold, double omega, double *J, double *K) {
    if (!P) return fail(JK_EINVAL, "plan is NULL");
    if (!D || nset < 1) return fail(JK_EINVAL, "D must be non-NULL and nset >= 1");
    const bool do_j = flags & JK_DO_J, do_k = flags & JK_DO_K;
    if (flags & ~(JK_DO_J | JK_DO_K | JK_ACCUMULATE | JK_CHECK_SYMMETRY | JK_DETERMINISTIC))
        return fail(JK_EINVAL, "unknown flag bits 0x%x", flags);
    if ((do_j && !J) || (do_k && !K)) return fail(JK_EINVAL, "J/K output missing for a requested matrix");
    if (precision != JK_FP64 && precision != JK_MIXED && precision != JK_FP32) return fail(JK_EINVAL, "bad precision %d", precision);
    if (precision == JK_MIXED && !(std::isfinite(mix_threshold) && mix_threshold >= 0.0)) return fail(JK_EINVAL, "mix_threshold must be finite and >= 0");
    if (!std::isfinite(omega)) return fail(JK_EINVAL, "omega must be finite");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev != P->device) return fail(JK_EINVAL, "plan was created on device %d, current device is %d", P->device, dev);
    return 0;
}

// max |D - D^T| and max |D| over every density, on the device; the host
// compares them (JK_CHECK_SYMMETRY).  out[0] = asymmetry, out[1] = largest.
__global__ void k_symmetry(const double *D, int n, int nset, unsigned long long *out) {
    const int64_t tot = (int64_t)nset * n * n;
    double asym = 0.0, big = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < tot; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = t / ((int64_t)n * n);
        const int i = (int)((t / n) % n), j = (int)(t % n);
        const double v = D[t];
        asym = fmax(asym, fabs(v - D[s * n * n + (int64_t)j * n + i]));
        // a non-finite entry makes the largest magnitude infinite
        big = fmax(big, isfinite(v) ? fabs(v) : INFINITY);
    }
    // non-negative doubles order like their bit patterns
    atomicMax(&out[0], (unsigned long long)__double_as_longlong(asym));
    atomicMax(&out[1], (unsigned long long)__double_as_longlong(big));
}

static int check_symmetry(const jk_plan *P, const double *D, int nset, hipStream_t s, unsigned long long *scratch2) {
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, scratch2, 2);
    hipLaunchKernelGGL(k_symmetry, dim3(grid_for((int64_t)nset * P->nao * P->nao, 256)), dim3(256), 0, s, D, P->nao, nset, scratch2);
    HIPCHK(hipGetLastError());
    unsigned long long h[2];
    HIPCHK(hipMemcpyAsync(h, scratch2, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double asym, big;
    std::memcpy(&asym, &h[0], sizeof asym);
    std::memcpy(&big, &h[1], sizeof big);
    if (!(std::isfinite(asym) && std::isfinite(big))) return fail(JK_EINVAL, "D holds non-finite values");
    if (asym > 1e-12 * big) return fail(JK_EINVAL, "D is not symmetric: max|D - D^T| = %.3e, max|D| = %.3e", asym, big);
    return 0;
}

// One J/K build into the given scratch (both entry points).
int execute_impl(jk_plan *P, const double *D, int32_t nset, int32_t flags, int32_t precision, double mix_threshold,
                        double omega, double *J, double *K, hipStream_t s, const Scratch &sc, bool allow_profile) {
    const bool do_j = flags & JK_DO_J, do_k = flags & JK_DO_K;
    const bool det = flags & JK_DETERMINISTIC;
    int rc;
    if (det && !sc.det) return fail(JK_EINVAL, "JK_DETERMINISTIC needs the plan's own scratch (jk_execute)");
    if ((flags & JK_CHECK_SYMMETRY) && (rc = check_symmetry(P, D, nset, s, sc.nsel))) return rc;
    const size_t m = (size_t)P->naoc * P->naoc;
    // accumulation targets: FP64 buffers, or in the fixed-order mode the
    // three limb buffers (J', K', pair-ordered J'), each 3 x detL elements
    double *const Jc = det ? sc.det : sc.Jc;
    double *const Kc = det ? sc.det + 3 * sc.detL : sc.Kc;
    double *const jpb = det ? sc.det + 6 * sc.detL : sc.jp;
    const double *Dc = D;
    if (P->sph) {
        hipLaunchKernelGGL(k_sph_to_cart, dim3(grid_for((int64_t)nset * m, 256)), dim3(256), 0, s, P->maps, D, sc.Dc, P->nao, P->naoc, nset);
        HIPCHK(hipGetLastError());
        Dc = sc.Dc;
    }
    if (det) {
        hipLaunchKernelGGL(k_fill, dim3(grid_for(9 * sc.detL, 256)), dim3(256), 0, s, sc.det, 9 * sc.detL, 0.0);
    } else {
        hipLaunchKernelGGL(k_fill, dim3(grid_for((int64_t)nset * m, 256)), dim3(256), 0, s, Jc, (int64_t)(nset * m), 0.0);
        hipLaunchKernelGGL(k_fill, dim3(grid_for((int64_t)nset * m, 256)), dim3(256), 0, s, Kc, (int64_t)(nset * m), 0.0);
        hipLaunchKernelGGL(k_fill, dim3(grid_for((int64_t)nset * P->njp, 256)), dim3(256), 0, s, jpb, (int64_t)nset * P->njp, 0.0);
    }
    const int nctr = (int)scratch_sizes(P, nset).nsel;
    hipLaunchKernelGGL(k_fill_u64, dim3((nctr + 255) / 256), dim3(256), 0, s, sc.nsel, nctr);
    HIPCHK(hipGetLastError());
    if (precision == JK_MIXED || P->dscreen > 0.0) {
        hipLaunchKernelGGL(k_dmax, dim3((P->ns * P->ns + 255) / 256), dim3(256), 0, s, Dc, P->maps.aoc, P->maps.l, P->ns, P->naoc, nset, sc.dmax);
        hipLaunchKernelGGL(k_dmax_all, dim3(1), dim3(256), 0, s, sc.dmax, P->ns);
        HIPCHK(hipGetLastError());
    }
    JkArgs a{};
    a.pairs = P->d_pairs;
    a.pp = P->d_pp;
    a.D = Dc;
    a.J = Jc;
    a.K = Kc;
    a.mstride = (int64_t)m;
    a.jp = jpb;
    a.det = det ? sc.detL : 0;
    a.jpstride = P->njp;
    a.nao = P->naoc;
    a.nset = nset;
    a.do_j = do_j;
    a.do_k = do_k;
    a.dmax = sc.dmax;
    a.nshell = P->ns;
    a.mix_thr = mix_threshold;
    a.omega = omega;
    a.dscreen = P->dscreen;
    a.tab = P->tab;
    a.tpos = P->d_tpos;
    a.aoc = P->maps.aoc;
    P->last_nsel = sc.nsel;
    P->last_precision = precision;
    P->last_fixed.assign(P->cls.size() * 8, 0);
    // with every quartet selected and no density screening a launch
    // evaluates exactly its quartets: no device counting
    const bool count_on_device = precision == JK_MIXED || P->dscreen > 0.0;
    auto set_count = [&](int slot, int64_t host_count) {
        a.nsel = count_on_device ? sc.nsel + (size_t)slot * NSEL_SLOTS * NSEL_STRIDE : nullptr;
        P->last_fixed[slot] = count_on_device ? -1 : host_count;
    };
    const bool profile = P->profile && allow_profile;
    // launches in order: timing slot of each
    std::vector<int> slots;
    int nev = 0;
    auto mark = [&](int slot) -> int {
        if (!profile) return 0;
        if ((int)P->events.size() <= nev) {
            hipEvent_t ev;
            HIPCHK(hipEventCreate(&ev));
            P->events.push_back(ev);
        }
        HIPCHK(hipEventRecord(P->events[nev++], s));
        if (slot >= 0) slots.push_back(slot);
        return 0;
    };
    // the class launches only add into Jc, Kc and jp with atomics, so
    // classes may overlap: each class goes whole to the least loaded of the
    // plan's streams (by model flops), forked from s and joined back into s
    // before the J'_KL scatter. Timed builds stay on s.
    const hipStream_t s0 = s;
    const int nst = profile ? 1 : P->nstream;
    double load[jk_plan::MAXSTREAM] = {};
    if (nst > 1) {
        HIPCHK(hipEventRecord(P->fork_ev, s0));
        for (int k = 1; k < nst; ++k) HIPCHK(hipStreamWaitEvent(P->streams[k], P->fork_ev, 0));
    }
    for (size_t ci = 0; ci < P->cls.size(); ++ci) {
        const ClassTask &c = P->cls[ci];
        const ClassEntry &e = g_classes[class_id(c.li, c.lj, c.lk, c.ll)];
        if (nst > 1) {
            int k = 0;
            for (int t = 1; t < nst; ++t)
                if (load[t] < load[k]) k = t;
            load[k] += c.flops;
            s = k == 0 ? s0 : P->streams[k];
        }
        a.ket_list = c.d_ket;
        a.same = c.same;
        a.npb = c.npb;
        a.npk = c.npk;
        a.nq = (int32_t)c.nq;
        // mixed: a single-precision pass over the quartets below the
        // threshold, then a double-precision pass over the rest; both walk
        // the class's tiles and row tasks
        const bool msplit = precision == JK_MIXED && c.split;  // (else the class runs in FP64)
        const int npass = msplit ? 2 : 1;
        for (int pass = 0; pass < npass; ++pass) {
            const int pr = msplit ? (pass == 0 ? 1 : 0) : (precision == JK_FP32 ? 1 : 0);
            a.sel = msplit ? (pass == 0 ? SEL_LO : SEL_HI) : SEL_ALL;
            a.dstage = 0;
            const int f = c.fam[pr];
            // tiles (the short rest) of family 3 classes run in the fallback family
            const int ft = f == 3 ? tile_fallback(c.li, c.lj, c.lk, c.ll) : f;
            const int slot = (int)(2 * ci + pr) * 4;  // + kind
            const int ncols = c.ncolK + (c.seg_same ? 0 : c.ncolL);
            // the double-precision pass of the mixed split runs as tiles: its
            // quartets are the first few kets of each bra (largest Schwarz
            // factors), a fraction of one row-mode pass per bra, and tiles
            // past them end at their first ket
            // (and every class in the fixed-order mode: the row kernels add
            // into their LDS rows from several waves, in no fixed order)
            const bool tiles_only = a.sel == SEL_HI || det;
            const bool longrows = !tiles_only && c.row_ok[pr] && c.nrow > 0 && e.row[f - 1][pr] &&
                                  row_lds_bytes(e, f, pr, c.li, c.lj, nset, ncols, 4, c.npb) <= (size_t)ROW_LDS_MAX && !P->no_row;
            const bool shortrows = !tiles_only && c.row_short[pr] && c.nsrow > 0 && e.srow[f - 1][pr] &&
                                   (longrows || c.nrow == 0) &&
                                   row_lds_bytes(e, f, pr, c.li, c.lj, nset, ncols, 1, c.npb) <= (size_t)ROW_LDS_MAX && !P->no_row;
            if (longrows || shortrows) {
                a.bra_list = c.d_bra;
                a.bra_cnt = c.d_cnt;
                a.tshK = c.d_tshK;
                a.tshL = c.d_tshL;
                a.ncolK = c.ncolK;
                a.ncolL = c.ncolL;
                a.seg_same = c.seg_same;
            }
            if (longrows) {
                // long bras: 256-lane workgroups over chunks of their kets;
                // family 1 stages the bra's D rows in LDS where the
                // workgroup's LDS stays within DSTAGE_LDS_MAX
                a.row_pos = c.d_rowc[f - 1];
                a.nrow = c.nrowc[f - 1];
                a.dstage = f == 1 && k1_dstage_class(c.li, c.lj) && !P->no_dstage &&
                           row_lds_bytes(e, f, pr, c.li, c.lj, nset, ncols, 4, c.npb) +
                                   sizeof(double) * (size_t)nset * (ncart(c.li) + ncart(c.lj)) * ncols <=
                               (size_t)DSTAGE_LDS_MAX;
                set_count(slot + 1, c.nq_row);
                if ((rc = mark(slot + 1))) return rc;
                HIPCHK(e.row[f - 1][pr](a, s));
            }
            if (shortrows) {
                // short bras: one 64-lane workgroup each
                a.dstage = 0;
                a.row_pos = c.d_srowt;
                a.nrow = c.nsrow;
                set_count(slot + 3, c.nq - c.nq_row);
                if ((rc = mark(slot + 3))) return rc;
                HIPCHK(e.srow[f - 1][pr](a, s));
                a.ntiles = 0;
            } else if (longrows) {
                // the short rest as tiles
                a.bra_list = c.d_sbra;
                a.bra_cnt = c.d_scnt;
                a.nbra = c.nsbra;
                a.tile_off = c.d_stile[ft - 1];
                a.ntiles = c.nstiles[ft - 1];
            } else {
                a.bra_list = c.d_bra;
                a.bra_cnt = c.d_cnt;
                a.nbra = c.nbra;
                a.tile_off = c.d_tile[ft - 1];
                a.ntiles = c.ntiles[ft - 1];
            }
            if (a.ntiles > 0) {
                set_count(slot, longrows ? c.nq - c.nq_row : c.nq);
                if ((rc = mark(slot))) return rc;
                HIPCHK(e.tiles[ft - 1][pr](a, s));
            }
        }
    }
    s = s0;
    for (int k = 1; k < nst; ++k) {
        HIPCHK(hipEventRecord(P->join_ev[k], P->streams[k]));
        HIPCHK(hipStreamWaitEvent(s0, P->join_ev[k], 0));
    }
    if (profile) {
        if ((rc = mark(-1))) return rc;
        HIPCHK(hipEventSynchronize(P->events[nev - 1]));
        std::vector<int64_t> cnt;
        if ((rc = launch_counts(P, &cnt))) return rc;
        for (size_t k = 0; k < slots.size(); ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, P->events[k], P->events[k + 1]));
            jk_class_timing &t = P->timing[slots[k]];
            const ClassTask &c = P->cls[slots[k] / 8];
            const int64_t nq = cnt[slots[k]];
            t.ms += ms;
            t.launches += 1;
            t.nquartets += nq;
            t.model_flops += c.flops * (double)nq / (double)c.nq;
        }
    }
    const int acc = (flags & JK_ACCUMULATE) ? 1 : 0;
    const int64_t mo = (int64_t)nset * P->nao * P->nao;
    const int npair = (int)P->hpairs.size();
    if (det) {
        const int64_t nm = (int64_t)nset * m, nj = (int64_t)nset * P->njp;
        hipLaunchKernelGGL(k_det_collapse, dim3(grid_for(nm, 256)), dim3(256), 0, s, Jc, sc.detL, nm);
        hipLaunchKernelGGL(k_det_collapse, dim3(grid_for(nm, 256)), dim3(256), 0, s, Kc, sc.detL, nm);
        hipLaunchKernelGGL(k_det_collapse, dim3(grid_for(nj, 256)), dim3(256), 0, s, jpb, sc.detL, nj);
    }
    if (do_j) {
        const int64_t nt = (int64_t)nset * npair * 64;
        hipLaunchKernelGGL(k_jp_scatter, dim3(grid_for(nt, 256)), dim3(256), 0, s, P->d_pairs, P->maps.l, jpb, P->njp,
                           Jc, (int64_t)m, P->naoc, npair, nt);
    }
    if (do_j) hipLaunchKernelGGL(k_finalize, dim3(grid_for(mo, 256)), dim3(256), 0, s, P->maps, Jc, J, P->nao, P->naoc, nset, P->sph, acc);
    if (do_k) hipLaunchKernelGGL(k_finalize, dim3(grid_for(mo, 256)), dim3(256), 0, s, P->maps, Kc, K, P->nao, P->naoc, nset, P->sph, acc);
    HIPCHK(hipGetLastError());
    return JK_OK;
}

extern "C" int jk_execute(jk_plan *P, const double *D, int32_t nset, int32_t flags, int32_t precision, double mix_threshold,
                          double omega, double *J, double *K, void *stream) {
    int rc = check_execute_args(P, D, nset, flags, precision, mix_threshold, omega, J, K);
    if (rc) return rc;
    Scratch sc;
    if ((rc = ensure_scratch(P, nset, &sc, (flags & JK_DETERMINISTIC) != 0))) return rc;
    return execute_impl(P, D, nset, flags, precision, mix_threshold, omega, J, K, (hipStream_t)stream, sc, true);
}

extern "C" int jk_plan_set_density_screening(jk_plan *P, double threshold) {
    if (!P) return fail(JK_EINVAL, "plan is NULL");
    if (!(std::isfinite(threshold) && threshold >= 0.0)) return fail(JK_EINVAL, "threshold must be finite and >= 0");
    P->dscreen = threshold;
    return JK_OK;
}

extern "C" int jk_plan_profile(jk_plan *P, int32_t enable) {
    if (!P) return fail(JK_EINVAL, "plan is NULL");
    P->profile = enable != 0;
    P->timing.assign(8 * P->cls.size(), jk_class_timing{});
    for (size_t ci = 0; ci < P->cls.size(); ++ci)
        for (int k = 0; k < 2; ++k)
            for (int kind = 0; kind < 4; ++kind) {
                const ClassTask &c = P->cls[ci];
                jk_class_timing &t = P->timing[(2 * ci + k) * 4 + kind];
                t.li = c.li; t.lj = c.lj; t.lk = c.lk; t.ll = c.ll;
                t.npb = c.npb; t.npk = c.npk;
                t.precision = (k && kind != 2) ? JK_FP32 : JK_FP64;
                // tiles of a family-3 class run in its fallback family
                t.family = kind == 0 && c.fam[k] == 3 ? tile_fallback(c.li, c.lj, c.lk, c.ll) : c.fam[k];
                t.kind = kind;
            }
    return 0;
}

extern "C" int jk_plan_timings(const jk_plan *P, jk_class_timing *out, int32_t cap, int32_t *count) {
    if (!P || !count || (cap > 0 && !out)) return fail(JK_EINVAL, "NULL argument");
    int n = 0;
    for (const jk_class_timing &t : P->timing) {
        if (t.launches == 0) continue;
        if (n < cap) out[n] = t;
        ++n;
    }
    *count = n;
    return 0;
}

extern "C" int jk_build(const jk_basis *basis, const double *D, int32_t nset, double cutoff, int32_t precision, double *J, double *K,
                        void *stream) {
    jk_plan *P = nullptr;
    int rc = jk_plan_create(basis, cutoff, &P);
    if (rc) return rc;
    rc = jk_execute(P, D, nset, JK_DO_J | JK_DO_K, precision, 1e-4, 0.0, J, K, stream);
    if (rc == 0) {
        hipError_t e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) rc = fail(JK_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    }
    jk_plan_destroy(P);
    return rc;
}

extern "C" int jk_eri_block(jk_plan *P, int32_t I, int32_t J, int32_t K, int32_t L, int32_t precision, double *host_out) {
    if (!P || !host_out) return fail(JK_EINVAL, "NULL argument");
    const int ns = P->ns;
    if (I < 0 || J < 0 || K < 0 || L < 0 || I >= ns || J >= ns || K >= ns || L >= ns) return fail(JK_EINVAL, "shell index out of range");
    if (precision != JK_FP64 && precision != JK_FP32) return fail(JK_EINVAL, "precision must be JK_FP64 or JK_FP32");
    int pb = P->pair_of[(size_t)I * ns + J], pk = P->pair_of[(size_t)K * ns + L];
    const PairRec &rb0 = P->hpairs[pb], &rk0 = P->hpairs[pk];
    auto lk = [&](const PairRec &r) { return std::make_pair(P->l[r.ish], P->l[r.jsh]); };
    bool swap = lk(rk0) > lk(rb0);
    if (swap) std::swap(pb, pk);
    const PairRec &rb = P->hpairs[pb], &rk = P->hpairs[pk];
    const int li = P->l[rb.ish], lj = P->l[rb.jsh], lk2 = P->l[rk.ish], ll = P->l[rk.jsh];
    const int ni = ncart(li), nj = ncart(lj), nk = ncart(lk2), nl = ncart(ll);
    int32_t *d_q;
    double *d_out;
    HIPCHK(hipMalloc(&d_q, 2 * sizeof(int32_t)));
    const int32_t qs[2] = {pb, pk};
    HIPCHK(hipMemcpy(d_q, qs, sizeof qs, hipMemcpyHostToDevice));
    HIPCHK(hipMalloc(&d_out, sizeof(double) * ni * nj * nk * nl));
    int rc = launch_export(P, li, lj, lk2, ll, precision, d_q, d_q + 1, 1, d_out, 0);
    std::vector<double> blk((size_t)ni * nj * nk * nl);
    if (!rc) {
        hipError_t e = hipMemcpy(blk.data(), d_out, sizeof(double) * blk.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = fail(JK_EDEVICE, "hipMemcpy: %s", hipGetErrorString(e));
    }
    (void)hipFree(d_q);
    (void)hipFree(d_out);
    if (rc) return rc;
    // blk is [a in rb.ish][b in rb.jsh][c in rk.ish][d in rk.jsh]; map to (I J | K L)
    const int sh[4] = {rb.ish, rb.jsh, rk.ish, rk.jsh};
    const int dims[4] = {ni, nj, nk, nl};
    const int want[4] = {I, J, K, L};
    // position of each requested index among the block axes
    int pos[4];
    {
        const int wb[2] = {swap ? K : I, swap ? L : J};
        const int wk[2] = {swap ? I : K, swap ? J : L};
        // bra block axes 0,1 hold (rb.ish, rb.jsh) == {wb[0], wb[1]} in some order
        int bpos0 = (rb.ish == wb[0]) ? 0 : 1;
        if (wb[0] == wb[1]) bpos0 = 0;
        int kpos0 = (rk.ish == wk[0]) ? 2 : 3;
        if (wk[0] == wk[1]) kpos0 = 2;
        const int bpos1 = 1 - bpos0, kpos1 = 5 - kpos0;
        if (!swap) { pos[0] = bpos0; pos[1] = bpos1; pos[2] = kpos0; pos[3] = kpos1; }
        else { pos[2] = bpos0; pos[3] = bpos1; pos[0] = kpos0; pos[1] = kpos1; }
    }
    (void)sh; (void)want;
    const int oi = dims[pos[0]], oj = dims[pos[1]], ok = dims[pos[2]], ol = dims[pos[3]];
    int strides[4] = {nj * nk * nl, nk * nl, nl, 1};
    for (int a = 0; a < oi; ++a)
        for (int b = 0; b < oj; ++b)
            for (int c = 0; c < ok; ++c)
                for (int d = 0; d < ol; ++d) {
                    int idx[4];
                    idx[pos[0]] = a; idx[pos[1]] = b; idx[pos[2]] = c; idx[pos[3]] = d;
                    host_out[((a * oj + b) * ok + c) * ol + d] =
                        blk[idx[0] * strides[0] + idx[1] * strides[1] + idx[2] * strides[2] + idx[3] * strides[3]];
                }
    return 0;
}

extern "C" int jk_rys_eval(int32_t n, const double *T, int32_t count, int32_t precision, double *roots, double *weights) {
    if (n < 1 || n > JKT_RYS_NMAX || count < 0 || (count > 0 && (!T || !roots || !weights))) return fail(JK_EINVAL, "bad arguments");
    if (precision != JK_FP64 && precision != JK_FP32) return fail(JK_EINVAL, "precision must be JK_FP64 or JK_FP32");
    for (int i = 0; i < count; ++i)
        if (!(std::isfinite(T[i]) && T[i] >= 0.0)) return fail(JK_EINVAL, "T must be finite and >= 0");
    if (count == 0) return 0;
    Tables tab;
    int rc = tables_for_device(&tab);
    if (rc) return rc;
    double *dT, *du, *dw;
    HIPCHK(hipMalloc(&dT, sizeof(double) * count));
    HIPCHK(hipMalloc(&du, sizeof(double) * count * n));
    HIPCHK(hipMalloc(&dw, sizeof(double) * count * n));
    HIPCHK(hipMemcpy(dT, T, sizeof(double) * count, hipMemcpyHostToDevice));
    const dim3 g((count + 127) / 128), b(128);
#define RYS_CASE(N)                                                                                       \
    case N:                                                                                               \
        if (precision == JK_FP64) hipLaunchKernelGGL((k_rys_eval<N, double>), g, b, 0, 0, tab, dT, count, du, dw); \
        else hipLaunchKernelGGL((k_rys_eval<N, float>), g, b, 0, 0, tab, dT, count, du, dw);              \
        break;
    switch (n) { RYS_CASE(1) RYS_CASE(2) RYS_CASE(3) RYS_CASE(4) RYS_CASE(5) RYS_CASE(6) RYS_CASE(7) RYS_CASE(8) RYS_CASE(9) }
#undef RYS_CASE
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy(roots, du, sizeof(double) * count * n, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(weights, dw, sizeof(double) * count * n, hipMemcpyDeviceToHost));
    (void)hipFree(dT); (void)hipFree(du); (void)hipFree(dw);
    return 0;
}

extern "C" int jk_boys_eval(int32_t mmax, const double *T, int32_t count, int32_t precision, double *out) {
    if (mmax != 1 || count < 0 || (count > 0 && (!T || !out))) return fail(JK_EINVAL, "bad arguments (m must be 1)");
    if (precision != JK_FP64 && precision != JK_FP32) return fail(JK_EINVAL, "precision must be JK_FP64 or JK_FP32");
    for (int i = 0; i < count; ++i)
        if (!(std::isfinite(T[i]) && T[i] >= 0.0)) return fail(JK_EINVAL, "T must be finite and >= 0");
    if (count == 0) return 0;
    Tables tab;
    int rc = tables_for_device(&tab);
    if (rc) return rc;
    double *dT, *dout;
    HIPCHK(hipMalloc(&dT, sizeof(double) * count));
    HIPCHK(hipMalloc(&dout, sizeof(double) * count * 2));
    HIPCHK(hipMemcpy(dT, T, sizeof(double) * count, hipMemcpyHostToDevice));
    if (precision == JK_FP64) hipLaunchKernelGGL((k_boys_eval<double>), dim3((count + 127) / 128), dim3(128), 0, 0, tab, dT, count, dout);
    else hipLaunchKernelGGL((k_boys_eval<float>), dim3((count + 127) / 128), dim3(128), 0, 0, tab, dT, count, dout);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpy(out, dout, sizeof(double) * count * 2, hipMemcpyDeviceToHost));
    (void)hipFree(dT); (void)hipFree(dout);
    return 0;
}

// batched builds: see jk_batch.hip
