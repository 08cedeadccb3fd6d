// jk_common.h -- data layouts shared by the host planner and the kernels.
#pragma once
#include <stdint.h>

#ifdef __HIPCC__
#define JK_HD __host__ __device__
#else
#define JK_HD
#endif

namespace jk {

constexpr int LMAX = 4;
constexpr int NCLS = (LMAX + 1) * (LMAX + 1) * (LMAX + 1) * (LMAX + 1);

JK_HD constexpr int ncart(int l) { return (l + 1) * (l + 2) / 2; }
JK_HD constexpr int nroots(int li, int lj, int lk, int ll) { return (li + lj + lk + ll) / 2 + 1; }
JK_HD constexpr int class_id(int li, int lj, int lk, int ll) { return ((li * (LMAX + 1) + lj) * (LMAX + 1) + lk) * (LMAX + 1) + ll; }

// Cartesian exponent of component idx of a shell with angular momentum l
// along axis (0 x, 1 y, 2 z); reversed lexicographic order.
JK_HD constexpr int cart_comp(int l, int idx, int axis) {
    int n = 0;
    for (int x = l; x >= 0; --x)
        for (int y = l - x; y >= 0; --y) {
            if (n == idx) return axis == 0 ? x : (axis == 1 ? y : l - x - y);
            ++n;
        }
    return 0;
}

// One oriented shell pair (I, J): the first shell has the higher (l, nprim)
// type.  64 bytes.
struct PairRec {
    int32_t ish, jsh;      // shell indices
    int32_t aoi, aoj;      // Cartesian AO offsets
    int32_t pp_off, npp;   // first primitive pair, count
    int32_t pp_stride;     // distance between its consecutive primitive pairs
                           // (= the number of pairs of its type)
    int32_t jp_off;        // its first element in the pair-ordered J' buffer;
                           // element e (= i * ncart(l_J) + j) at jp_off + e * pp_stride
    double ab[3];          // A - B
    double q;              // Schwarz factor sqrt(max |(ab|ab)|)
};

// One primitive pair (a on A, b on B).  80 bytes.
struct PrimPair {
    double p;       // a + b
    double h;       // 1 / (2p)
    double kp;      // c_a c_b exp(-ab/p |AB|^2) / p
    double pad;
    double P[3];    // (a A + b B) / p
    double PA[3];   // P - A
};

// Kernel families per angular class (all that fit are built; the planner
// picks one per class and precision from the tuning table):
//   1: one lane per quartet (register-resident integral block);
//   2: a lane group per quartet, 2-D integrals staged in LDS.
JK_HD constexpr int ncart4(int li, int lj, int lk, int ll) { return ncart(li) * ncart(lj) * ncart(lk) * ncart(ll); }
JK_HD constexpr bool has_family1(int li, int lj, int lk, int ll) { return ncart4(li, lj, lk, ll) <= 180; }
JK_HD constexpr bool has_family2(int li, int lj, int lk, int ll) { return ncart4(li, lj, lk, ll) >= 18; }
JK_HD constexpr int default_family(int li, int lj, int lk, int ll) { return ncart4(li, lj, lk, ll) <= 36 ? 1 : 2; }
//   3: a lane per Cartesian component of the bra's first shell, each lane's
//      elements in registers, the vertical-recurrence tables in LDS (row
//      mode only; bras with short ket prefixes fall back to the tiles of
//      family 2, or 1 where 2 is not built).
JK_HD constexpr bool has_family3(int li, int lj, int lk, int ll) {
    return li >= 1 && ncart(lj) * ncart(lk) * ncart(ll) <= 64 && ncart4(li, lj, lk, ll) >= 27;
}
JK_HD constexpr int k3_qw(int li) { return 64 / ncart(li); }
// Family-1 row kernels that can stage the bra's D rows in LDS: the small
// bras, whose rows fit the staging budget on molecules of interest.
JK_HD constexpr bool k1_dstage_class(int li, int lj) { return ncart(li) + ncart(lj) <= 7; }
JK_HD constexpr int tile_fallback(int li, int lj, int lk, int ll) { return has_family2(li, lj, lk, ll) ? 2 : 1; }
// Family 2: lanes per quartet = ncart(li) * ncart(lk) (slot = (a, c)).
JK_HD constexpr int k2_slots(int li, int lj, int lk, int ll) { return ncart(li) * ncart(lk); }
JK_HD constexpr int k2_qw(int li, int lj, int lk, int ll) {
    return k2_slots(li, lj, lk, ll) >= 64 ? 1 : 64 / k2_slots(li, lj, lk, ll);
}

// Row mode: kets per workgroup task.  Long bras are cut into chunks so one
// bra's kets spread over several workgroups (family 1 computes 256 kets
// per pass, family 2 four waves of k2_qw quartets).
JK_HD constexpr int row_chunk(int fam, int li, int lj, int lk, int ll) {
    return fam == 1 ? 2048 : fam == 2 ? 256 * k2_qw(li, lj, lk, ll) : 256 * k3_qw(li);
}
// Quartets per wave-tile of a family.
JK_HD constexpr int quartets_per_tile(int fam, int li, int lj, int lk, int ll) {
    return fam == 1 ? 64 : k2_qw(li, lj, lk, ll);
}

// Quartet sources: tiles of (bra, Q-sorted ket prefix), or an explicit
// list whose blocks are written out (Schwarz diagonal, test hook).
enum { MODE_JK = 0, MODE_EXPORT = 1 };
// Row mode (family 1): one workgroup per bra with a long ket prefix; K rows
// of the bra's two shells accumulate in LDS over column-compressed segments
// (the columns of the ket shell types only) and are flushed once.
// Quartet selection of a launch: every quartet, or one side of the mixed
// precision split by the bound Q_IJ Q_KL max|D_block| against the threshold
// (SEL_LO: below it, the single-precision pass; SEL_HI: at or above it, the
// double-precision pass).  Both passes walk the same tiles and row tasks and
// mask the other side's lanes; a wave with no selected lane skips the work.
enum { SEL_ALL = 0, SEL_LO = 1, SEL_HI = 2 };
constexpr int NSEL_SLOTS = 16, NSEL_STRIDE = 8;  // counters per launch, 64 bytes apart

struct Tables {
    const double *rys;     // degree-major Rys fits, FP64
    const float *rys32;    // same, FP32
    const double *hx2, *hw;  // large-T Gauss-Hermite limit
    const float *hx2_32, *hw32;
    const double *boys;    // F_m on the T grid
    const float *boys32;
    const double *mom;     // [e^-T, F_3..F_9] on the T grid (two-root rule)
};

struct JkArgs {
    const PairRec *pairs;
    const PrimPair *pp;
    // JK mode: tiles over (bra list position, ket chunk)
    const int32_t *bra_list, *ket_list, *bra_cnt, *tile_off;
    int32_t nbra, ntiles, same, npb, npk;
    // EXPORT mode: explicit quartets
    const int32_t *q_bra, *q_ket;
    int32_t nq;
    double *out;
    // quartets this launch evaluated (after the selection and the density
    // screening): NSEL_SLOTS counters NSEL_STRIDE apart, picked by workgroup,
    // so that the waves of a launch do not all add to one address; NULL when
    // the host knows the count (every quartet selected, no density screening)
    unsigned long long *nsel;
    // row mode: tasks (list position, ket begin, ket end); column segments of the ket
    // shell types (shells of each type in order; tpos = index of a shell
    // within its type); segment L aliases segment K when the types match
    const int32_t *row_pos;
    int32_t nrow;
    const int32_t *tpos, *tshK, *tshL, *aoc;
    int32_t ncolK, ncolL, seg_same;
    // family-1 row mode: the bra's rows of D over the same compressed
    // columns are staged in LDS once per task (1), so the exchange digestion
    // reads them there instead of four scattered global loads per element
    int32_t dstage;
    // fixed-order accumulation (JK_DETERMINISTIC): J, K and jp each hold
    // three 64-bit integer limbs per element, det elements apart (0: FP64
    // atomics)
    int64_t det;
    // densities and results (Cartesian, [nset][nao][nao])
    const double *D;
    double *J, *K;
    int64_t mstride;
    // J'_KL of the ket pairs, pair-ordered ([nset][jpstride], see PairRec):
    // the lanes of a wave hold consecutive kets, so these atomics land on
    // consecutive addresses; added into J after the class kernels
    double *jp;
    int64_t jpstride;
    int32_t nao, nset, do_j, do_k;
    // precision split
    const double *dmax;  // [nshell][nshell] max |D| over the block and densities, then
                         // the largest entry of all (element nshell * nshell)
    int32_t nshell, sel;
    double mix_thr;
    // operator: 0 Coulomb, > 0 erf(omega r)/r, < 0 erfc(|omega| r)/r
    double omega;
    // density screening threshold on Q_IJ Q_KL max|D_block| (0: off)
    double dscreen;
    Tables tab;
};

}  // namespace jk
