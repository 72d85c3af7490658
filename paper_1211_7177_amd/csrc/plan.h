// Plan object: the octree, translation operators, correction blocks and the
// matvec workspace of one wavenumber.  Internal to the library.
#pragma once

#include <array>
#include <memory>
#include <vector>

#include "common.h"

namespace fmb {

constexpr int MAX_DEPTH = 10;
constexpr int MAX_ORDER = 24;
constexpr int NBITS = 21;
constexpr int N_M2L_OPS = 343;    // (dx,dy,dz) in [-3,3]^3, slot (dx+3)*49+(dy+3)*7+(dz+3); 316 used

struct Level {
    int64_t nbox = 0;
    DevBuf keys;          // u64[nbox]
    DevBuf start;         // i32[nbox+1] node range in Morton order
    DevBuf parent;        // i32[nbox]
    DevBuf center;        // f64[nbox][3]
    DevBuf nbr;           // i32[nbox][27]
    DevBuf child_start;   // i32[nbox+1] children (at level+1) ranges
    DevBuf octant;        // i32[nbox] child position in its parent (0..7)
    // far field (levels >= 2)
    int64_t nff = 0;
    int64_t slot_base = 0;   // first S|R slot of this level in the slot buffer
    DevBuf ff_ofs;        // i32[nbox+1]
    DevBuf ff_src;        // i32[nff]
    DevBuf ff_op;         // i32[nff] op slot 0..342
    DevBuf ff_by_op;      // i32[nff] entry ids grouped by op
    std::vector<int32_t> op_start;   // host, N_M2L_OPS+1
    // boxes of this level grouped by octant (for the M2M / L2L GEMMs)
    DevBuf by_octant;     // i32[nbox]
    std::array<int32_t, 9> oct_start{};
    // GEMM work tiles (op, first entry, count) for the translations into this level
    DevBuf tiles_m2l, tiles_m2m, tiles_l2l;
    int64_t ntiles_m2l = 0, ntiles_m2m = 0, ntiles_l2l = 0;
    // operators (precision of the plan), complex [op][P2 (dst)][P2 (src)]
    DevBuf m2l;           // [N_M2L_OPS] slots (unused slots left untouched)
    DevBuf m2m;           // [8]: child (level+1) octant -> this level
    DevBuf l2l;           // [8]: parent (level-1) -> child at this level with octant o
    // split-BF16 fragment-major copies of the three operator sets (FP32 plans only)
    DevBuf m2l_hi, m2l_lo, m2m_hi, m2m_lo, l2l_hi, l2l_lo;
    // expansions [nbox][nrhs_max][3][P2] complex (P2 = p^2 of this level)
    DevBuf M, L;
    // plans with an order per level (rotation / coaxial translations, hf.hip)
    int p = 0;                  // truncation order of this level
    DevBuf hW;                  // M2L rotation tables [polar-angle class][hwsz], plan precision
    DevBuf hWo;                 // octant rotation tables [2][hwszo] (cos theta = +-1/sqrt 3)
    DevBuf hph, hpho;           // e^{i m phi}: [343 offsets][p] and [16 octant directions][hpwo]
    DevBuf hC, hCss, hCrr;      // coaxial S|R [distance class][hcsz]; S|S from level+1; R|R from level-1
    DevBuf hopi;                // i32[343][2]: polar-angle class, distance class of each far-field offset
    DevBuf hboct;               // i32[16]: polar-angle class of each octant direction
    int64_t hwsz = 0, hwszo = 0, hcsz = 0;
    int hpwo = 0;
    DevBuf hoinfo;              // i32[16][2]: polar-angle class (and distance class 0) of each octant direction
    // chunk boundaries of the pipelined launches: degrees n < p, and |m| < p for the
    // coaxial shifts of the S|R set, of the S|S set into this level and of the R|R set into it
    DevBuf hnck, hmck, hmck_ss, hmck_rr;
    int hnnck = 0, hnmck = 0, hnmck_ss = 0, hnmck_rr = 0;
    int hnck_max = 0, hmck_max = 0, hmck_ss_max = 0, hmck_rr_max = 0;   // largest chunk (coefficients)
};

// stage timers (HIP events on the matvec stream), enabled per plan
enum Stage { ST_GATHER = 0, ST_P2M, ST_M2M, ST_M2L, ST_L2L, ST_L2P, ST_P2P, ST_CORR, ST_SCATTER, ST_SUMS, ST_M2L_FINE, ST_COUNT };

struct StageTimer {
    uint32_t mask = 0;                   // stages (bit 1 << stage) that record events
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[ST_COUNT];
    std::vector<int> pending_nk[ST_COUNT];   // kernel launches inside each bracket
    std::vector<hipEvent_t> pool;
    double ms[ST_COUNT] = {0};
    int64_t launches[ST_COUNT] = {0};
    hipEvent_t get();
    void begin(int st, hipStream_t s, hipEvent_t &e0);
    void end(int st, hipStream_t s, hipEvent_t e0, int nk = 1);
    void collect();
    void reset();
    ~StageTimer();
};

struct Plan {
    bool fuse_p2p = false;      // set by the two-product runner: the P2P step is left to its fused launch
    int64_t n = 0;
    int depth = 0, order = 0, P2 = 0, precision = FMB_FP64, nrhs_max = 1, corr_mode = 0;
    double k_re = 0, k_im = 0;
    double lo[3] = {0, 0, 0}, ext = 0;
    int64_t ntri = 0, tri_m = 1;
    int64_t p2p_pairs = 0;
    int leaf_target = 32;
    int translate_mode = FMB_TRANSLATE_FP32;
    // lossy wavenumbers: levels below far_lmin keep no far field (depth + 1: local only); a
    // local-only plan also drops near pairs with R^2 > rcut2
    double far_cutoff = 0.0;
    int far_lmin = 2;
    double rcut2 = 1e300;
    bool far_on() const { return far_lmin <= depth; }
    // order <= 0 at fmm_plan: an order per level for the tolerance `tol`, translations by
    // rotation and coaxial shift (order = the leaf level's order)
    bool hf = false;
    double tol = 0.0;
    DevBuf hscratch;  // vectors of translation stages too large for LDS
    DevBuf hX1, hX2;  // per-pair vectors of the pipelined translations (large orders)
    std::vector<Level> lv;
    // per-node data in Morton order
    DevBuf codes;     // u64[n] user order
    DevBuf perm;      // i32[n] Morton position -> user index
    DevBuf iperm;     // i32[n] user index -> Morton position
    DevBuf spts;      // f64[n][3]
    DevBuf snrm;      // f64[n][3]
    DevBuf sw;        // f64[n]
    DevBuf stri;      // i32[n]
    DevBuf inv_alpha; // f64[depth+1][order] 1/alpha_n per level
    DevBuf btab;      // basis recurrence constants in the plan's precision (BasisTab layout, N = order)
    DevBuf bgix;      // i32[order^2][7] R-table indices of the gradient terms
    // corrections (user order)
    DevBuf point_tri; // i32[n]
    DevBuf unrm;      // f64[n][3] normals, user order
    DevBuf tri_nodes; // i32[ntri][tri_m]
    DevBuf corr_v;    // c128[n][tri_m][3]
    DevBuf corr_g;    // c128[n][tri_m]
    // matvec workspace
    DevBuf src;       // [nrhs_max][n][7] complex (w a, w b, w n.a) in Morton order
    DevBuf ys;        // [nrhs_max][n][3] complex, Morton order
    DevBuf ybuf;      // GEMM output slots, largest level
    DevBuf aws;       // adjoint: [nrhs_max][n][12] potentials and gradients per channel, Morton order (on first use)
    DevBuf agath;     // adjoint: per R-table entry, the gradient terms that land on it (on first use)
    StageTimer timer;
    size_t device_bytes() const;
};

// plan-building steps (plan.hip)
// host_tri (optional, host i32[n]): triangle of each node; depths at which two
// nodes of one triangle fall in non-neighbouring leaves are refused (an
// automatic depth steps down instead)
void build_tree(Plan &P, const double *d_pts, hipStream_t s, const int32_t *host_tri = nullptr);
void gather_nodes(Plan &P, const double *d_pts, const double *d_nrm, const double *d_w, const int32_t *d_tri,
                  hipStream_t s);
void build_operators(Plan &P, hipStream_t s);
void build_basis_tables(Plan &P, hipStream_t s);
// order per level (hf.hip)
int hf_order(double kabs, double side, double tol);
void build_hf(Plan &P, hipStream_t s);
template <typename T> void hf_m2m(Plan &P, int l, int nrhs, hipStream_t s);
template <typename T> void hf_m2l(Plan &P, int l, int nrhs, hipStream_t s);
template <typename T> void hf_l2l(Plan &P, int l, int nrhs, hipStream_t s);
void build_corrections(Plan &P, const double *d_pts, const double *d_nrm, const double *d_tri,
                       hipStream_t s);
void scatter_with_corrections(Plan &P, const void *ys, const void *a, const void *b, void *y, int nrhs,
                              hipStream_t s);
// matvec (matvec.hip)
void run_matvec(Plan &P, const void *a, const void *b, void *y, int nrhs, hipStream_t s);
// the adjoint product (a_bar, b_bar) = Op^H y (adjoint.hip for its own steps)
void adjoint_prepare(Plan &P);
void adjoint_gather(Plan &P, const void *y, int nrhs, hipStream_t s);
void adjoint_l2p(Plan &P, int nrhs, hipStream_t s);
void adjoint_p2p(Plan &P, int nrhs, hipStream_t s);
void adjoint_finish(Plan &P, const void *y, void *abar, void *bbar, int nrhs, hipStream_t s);
void run_matvec_adjoint(Plan &P, const void *y, void *abar, void *bbar, int nrhs, hipStream_t s);
// two products, P0 on s0 and P1 on s1, their launches issued alternately
void run_matvec_pair(Plan &P0, const void *a0, const void *b0, void *y0, hipStream_t s0, Plan &P1, const void *a1,
                     const void *b1, void *y1, hipStream_t s1, int nrhs);

}  // namespace fmb

struct fmb_plan_s {
    fmb::Plan p;
};
