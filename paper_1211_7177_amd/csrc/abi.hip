// C entry points of the fmbem library: argument validation on the host,
// device uploads, and dispatch to the plan / matvec steps.
#include <algorithm>
#include <cstring>
#include <limits>

#include "plan.h"

namespace fmb {

thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

size_t Plan::device_bytes() const {
    size_t b = codes.bytes + perm.bytes + iperm.bytes + spts.bytes + snrm.bytes + sw.bytes + stri.bytes +
               inv_alpha.bytes + btab.bytes + bgix.bytes + point_tri.bytes + unrm.bytes + tri_nodes.bytes + corr_v.bytes + corr_g.bytes +
               src.bytes + ys.bytes + ybuf.bytes + hscratch.bytes + hX1.bytes + hX2.bytes;
    for (const Level &V : lv)
        b += V.keys.bytes + V.start.bytes + V.parent.bytes + V.center.bytes + V.nbr.bytes + V.child_start.bytes +
             V.octant.bytes + V.ff_ofs.bytes + V.ff_src.bytes + V.ff_op.bytes + V.ff_by_op.bytes + V.by_octant.bytes +
             V.m2l.bytes + V.m2m.bytes + V.l2l.bytes + V.m2l_hi.bytes + V.m2l_lo.bytes + V.m2m_hi.bytes +
             V.m2m_lo.bytes + V.l2l_hi.bytes + V.l2l_lo.bytes + V.M.bytes + V.L.bytes + V.tiles_m2l.bytes + V.tiles_m2m.bytes +
             V.tiles_l2l.bytes + V.hW.bytes + V.hWo.bytes + V.hph.bytes + V.hpho.bytes + V.hC.bytes + V.hCss.bytes +
             V.hCrr.bytes + V.hopi.bytes + V.hboct.bytes + V.hoinfo.bytes + V.hnck.bytes + V.hmck.bytes;
    return b;
}

void build_tiles(Plan &P, hipStream_t s);
void split_operators(Plan &P, hipStream_t s);
void alloc_workspace(Plan &P);

// Far-field levels kept for a lossy wavenumber: level l is kept while the
// damping exp(-Im k h_l) over its box side h_l (the least distance between two
// of its far-field boxes) stays at or above the cutoff.  h_l halves per level,
// so the kept levels are far_lmin..depth.
static void set_far_cutoff(Plan &P, double cutoff) {
    if (cutoff == 0.0) cutoff = P.precision == FMB_FP64 ? 1e-16 : 1e-8;
    P.far_cutoff = cutoff;
    P.far_lmin = 2;
    P.rcut2 = std::numeric_limits<double>::infinity();
    if (cutoff < 0.0 || P.k_im <= 0.0) return;
    const double decay = std::log(1.0 / cutoff);      // exp(-decay) = cutoff
    int l = 2;
    while (l <= P.depth && P.k_im * (P.ext / (double)(1 << l)) > decay) ++l;
    P.far_lmin = l;
    if (!P.far_on()) {
        const double rc = decay / P.k_im;
        P.rcut2 = rc * rc;
    }
}

static void upload(DevBuf &d, const void *h, size_t bytes, hipStream_t s) {
    d.alloc(bytes);
    FMB_CHECK_HIP(hipMemcpyAsync(d.p, h, bytes, hipMemcpyHostToDevice, s));
}

}  // namespace fmb

using namespace fmb;

extern "C" {

const char *fmb_last_error(void) { return g_last_error.c_str(); }

int fmb_plan_opts_default(fmb_plan_opts *o) {
    if (!o) return FMB_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->depth = 0;
    o->precision = FMB_FP64;
    o->nrhs_max = 1;
    o->corr_mode = FMB_CORR_LINEAR;
    o->leaf_target = 32;
    return FMB_OK;
}

int fmm_plan(const double *points, const double *normals, const double *weights, int64_t n, double k_re,
             double k_im, int32_t order, const fmb_plan_opts *opts, void *stream, fmb_plan_t *out) {
    return guarded([&] {
        FMB_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        FMB_REQUIRE(points && normals && weights, "points, normals and weights are required");
        FMB_REQUIRE(n >= 2 && n < (int64_t)1 << 30, "n must be in [2, 2^30)");
        FMB_REQUIRE(std::isfinite(k_re) && std::isfinite(k_im) && k_im >= 0.0, "k must be finite with Im k >= 0");
        FMB_REQUIRE(k_re != 0.0 || k_im != 0.0, "k must be non-zero");
        FMB_REQUIRE(order <= MAX_ORDER, "order must be <= 24 (or <= 0: an order per level for opts->tol)");
        fmb_plan_opts o;
        fmb_plan_opts_default(&o);
        if (opts) o = *opts;
        FMB_REQUIRE(o.depth == 0 || (o.depth >= 2 && o.depth <= MAX_DEPTH), "depth must be 0 or in [2, 10]");
        FMB_REQUIRE(o.precision == FMB_FP64 || o.precision == FMB_FP32, "precision must be FMB_FP64 or FMB_FP32");
        FMB_REQUIRE(o.nrhs_max >= 1 && o.nrhs_max <= 1024, "nrhs_max must be in [1, 1024]");
        FMB_REQUIRE(o.corr_mode >= 0 && o.corr_mode <= 2, "corr_mode must be 0, 1 or 2");
        for (int64_t i = 0; i < 3 * n; ++i) {
            FMB_REQUIRE(std::isfinite(points[i]), "non-finite point coordinate");
            FMB_REQUIRE(std::isfinite(normals[i]), "non-finite normal component");
        }
        for (int64_t i = 0; i < n; ++i) {
            const double *v = normals + 3 * i;
            double l2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
            FMB_REQUIRE(std::fabs(std::sqrt(l2) - 1.0) <= 1e-6, "normal " + std::to_string(i) + " is not unit length");
            FMB_REQUIRE(std::isfinite(weights[i]) && weights[i] > 0.0, "weights must be finite and positive");
        }
        {
            // coincident points would meet at R = 0 in the near field: refuse them
            std::vector<int64_t> idx(n);
            for (int64_t i = 0; i < n; ++i) idx[i] = i;
            std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
                return std::lexicographical_compare(points + 3 * a, points + 3 * a + 3, points + 3 * b,
                                                    points + 3 * b + 3);
            });
            for (int64_t i = 1; i < n; ++i) {
                const double *p = points + 3 * idx[i], *q = points + 3 * idx[i - 1];
                FMB_REQUIRE(!(p[0] == q[0] && p[1] == q[1] && p[2] == q[2]),
                            "duplicate points " + std::to_string(idx[i - 1]) + " and " + std::to_string(idx[i]));
            }
        }
        std::vector<int32_t> tri;
        int64_t ntri = 0;
        if (o.point_tri) {
            FMB_REQUIRE(o.ntri >= 1, "ntri must be >= 1 when point_tri is given");
            tri.assign(o.point_tri, o.point_tri + n);
            for (int64_t i = 0; i < n; ++i)
                FMB_REQUIRE(tri[i] >= 0 && tri[i] < o.ntri, "point_tri entry out of range");
            ntri = o.ntri;
        } else {
            FMB_REQUIRE(o.corr_mode == FMB_CORR_NONE, "self-triangle corrections need point_tri and tri_vertices");
            tri.resize(n);
            for (int64_t i = 0; i < n; ++i) tri[i] = (int32_t)i;
            ntri = n;
        }
        int64_t m = 1;
        if (o.corr_mode != FMB_CORR_NONE) {
            FMB_REQUIRE(o.tri_vertices != nullptr, "corr_mode > 0 needs tri_vertices");
            FMB_REQUIRE(n % ntri == 0 && (n / ntri == 1 || n / ntri == 3),
                        "every triangle must hold 1 or 3 nodes (n / ntri in {1, 3})");
            m = n / ntri;
            for (int64_t i = 0; i < 9 * ntri; ++i) FMB_REQUIRE(std::isfinite(o.tri_vertices[i]), "non-finite vertex");
        }
        hipStream_t s = (hipStream_t)stream;
        auto *h = new fmb_plan_s;
        std::unique_ptr<fmb_plan_s> guard(h);
        Plan &P = h->p;
        P.n = n;
        P.depth = o.depth;
        P.hf = order <= 0;
        if (P.hf) {
            P.tol = o.tol > 0.0 ? o.tol : (o.precision == FMB_FP64 ? 1e-6 : 1e-4);
            FMB_REQUIRE(P.tol < 1.0 && P.tol >= 1e-15, "tol must be in [1e-15, 1)");
        }
        P.order = order;
        P.P2 = order * order;
        P.precision = o.precision;
        P.nrhs_max = o.nrhs_max;
        P.corr_mode = o.corr_mode;
        P.k_re = k_re;
        P.k_im = k_im;
        P.ntri = ntri;
        P.tri_m = m;
        P.leaf_target = o.leaf_target > 0 ? o.leaf_target : 32;
        FMB_REQUIRE(o.translate_mode >= 0 && o.translate_mode <= 2, "translate_mode must be 0, 1 or 2");
        P.translate_mode = o.translate_mode == FMB_TRANSLATE_BF16X3 ? FMB_TRANSLATE_BF16X3 : FMB_TRANSLATE_FP32;
        DevBuf d_pts, d_nrm, d_w, d_tv;
        upload(d_pts, points, n * 3 * sizeof(double), s);
        upload(d_nrm, normals, n * 3 * sizeof(double), s);
        upload(d_w, weights, n * sizeof(double), s);
        upload(P.point_tri, tri.data(), n * sizeof(int32_t), s);
        upload(P.unrm, normals, n * 3 * sizeof(double), s);
        build_tree(P, d_pts.as<double>(), s, ntri > 0 ? tri.data() : nullptr);
        set_far_cutoff(P, o.far_cutoff);
        gather_nodes(P, d_pts.as<double>(), d_nrm.as<double>(), d_w.as<double>(), P.point_tri.as<int32_t>(), s);
        if (P.hf) {
            // an order per level for the tolerance (its box size and the wavenumber)
            const double kabs = std::sqrt(k_re * k_re + k_im * k_im);
            for (int l = 0; l <= P.depth; ++l)
                P.lv[l].p = l >= std::max(2, P.far_lmin) ? hf_order(kabs, P.ext / (double)(1 << l), P.tol) : 0;
            P.order = P.far_on() ? P.lv[P.depth].p : 1;
            P.P2 = P.order * P.order;
            FMB_REQUIRE(P.order <= 40, "the leaf level needs an order above 40: choose a deeper octree");
            for (int l = 0; l <= P.depth; ++l)
                FMB_REQUIRE(P.lv[l].p <= 400, "a level needs an order above 400: boxes too large in wavelengths");
            build_basis_tables(P, s);
            if (P.far_on()) build_hf(P, s);
        } else {
            for (int l = 0; l <= P.depth; ++l) P.lv[l].p = order;
            build_operators(P, s);
            build_tiles(P, s);
            split_operators(P, s);
        }
        alloc_workspace(P);
        if (P.corr_mode != FMB_CORR_NONE) {
            upload(d_tv, o.tri_vertices, ntri * 9 * sizeof(double), s);
            build_corrections(P, d_pts.as<double>(), d_nrm.as<double>(), d_tv.as<double>(), s);
        }
        FMB_CHECK_HIP(hipStreamSynchronize(s));
        *out = guard.release();
    });
}

int fmm_matvec(fmb_plan_t plan, const void *a, const void *b, void *y, int32_t nrhs, void *stream) {
    return guarded([&] {
        FMB_REQUIRE(plan != nullptr, "plan is NULL");
        FMB_REQUIRE(a && b && y, "a, b and y are required");
        FMB_REQUIRE(y != a && y != b, "y must not alias a or b");
        FMB_REQUIRE(nrhs >= 1 && nrhs <= plan->p.nrhs_max, "nrhs must be in [1, nrhs_max]");
        run_matvec(plan->p, a, b, y, nrhs, (hipStream_t)stream);
    });
}

int fmm_matvec_adjoint(fmb_plan_t plan, const void *y, void *a_bar, void *b_bar, int32_t nrhs, void *stream) {
    return guarded([&] {
        FMB_REQUIRE(plan != nullptr, "plan is NULL");
        FMB_REQUIRE(y && a_bar && b_bar, "y, a_bar and b_bar are required");
        FMB_REQUIRE(a_bar != y && b_bar != y && a_bar != b_bar, "a_bar, b_bar and y must not alias");
        FMB_REQUIRE(nrhs >= 1 && nrhs <= plan->p.nrhs_max, "nrhs must be in [1, nrhs_max]");
        run_matvec_adjoint(plan->p, y, a_bar, b_bar, nrhs, (hipStream_t)stream);
    });
}

int fmm_plan_info(fmb_plan_t plan, fmb_plan_info *info) {
    return guarded([&] {
        FMB_REQUIRE(plan && info, "plan and info are required");
        const Plan &P = plan->p;
        std::memset(info, 0, sizeof(*info));
        info->depth = P.depth;
        info->order = P.order;
        info->precision = P.precision;
        info->nrhs_max = P.nrhs_max;
        info->n = P.n;
        for (int l = 0; l <= P.depth && l < 16; ++l) {
            info->nbox[l] = P.lv[l].nbox;
            info->m2l_pairs[l] = l >= std::max(2, P.far_lmin) ? P.lv[l].nff : 0;
            info->order_level[l] = P.lv[l].p;
        }
        info->far_lmin = P.far_lmin;
        info->p2p_pairs = P.p2p_pairs;
        info->corr_blocks = P.corr_mode ? P.n * P.tri_m : 0;
        info->device_bytes = (int64_t)P.device_bytes();
    });
}

int fmm_plan_export_tree(fmb_plan_t plan, int32_t level, uint64_t *codes, int32_t *perm, uint64_t *keys,
                         int32_t *parent, int32_t *start, int32_t *nbr, int32_t *ff_ofs, int32_t *ff_idx) {
    return guarded([&] {
        FMB_REQUIRE(plan != nullptr, "plan is NULL");
        const Plan &P = plan->p;
        FMB_REQUIRE(level >= 0 && level <= P.depth, "level out of range");
        const Level &V = P.lv[level];
        auto d2h = [](void *h, const DevBuf &d, size_t bytes) {
            if (h && bytes) FMB_CHECK_HIP(hipMemcpy(h, d.p, bytes, hipMemcpyDeviceToHost));
        };
        FMB_CHECK_HIP(hipDeviceSynchronize());
        d2h(codes, P.codes, P.n * sizeof(uint64_t));
        d2h(perm, P.perm, P.n * sizeof(int32_t));
        d2h(keys, V.keys, V.nbox * sizeof(uint64_t));
        d2h(parent, V.parent, V.nbox * sizeof(int32_t));
        d2h(start, V.start, (V.nbox + 1) * sizeof(int32_t));
        d2h(nbr, V.nbr, V.nbox * 27 * sizeof(int32_t));
        if (level >= 2) {
            d2h(ff_ofs, V.ff_ofs, (V.nbox + 1) * sizeof(int32_t));
            d2h(ff_idx, V.ff_src, V.nff * sizeof(int32_t));
        } else if (ff_ofs) {
            std::memset(ff_ofs, 0, (V.nbox + 1) * sizeof(int32_t));
        }
    });
}

int fmm_plan_profile(fmb_plan_t plan, int32_t mask) {
    return guarded([&] {
        FMB_REQUIRE(plan != nullptr, "plan is NULL");
        plan->p.timer.mask = (mask == 1) ? FMB_PROFILE_ALL : (uint32_t)mask & FMB_PROFILE_ALL;
    });
}

static_assert(ST_COUNT == FMB_NSTAGES, "stage list and FMB_NSTAGES differ");

int fmm_plan_profile_read(fmb_plan_t plan, double *ms, int64_t *launches, int32_t reset) {
    return guarded([&] {
        FMB_REQUIRE(plan != nullptr, "plan is NULL");
        StageTimer &t = plan->p.timer;
        t.collect();
        for (int i = 0; i < ST_COUNT; ++i) {
            if (ms) ms[i] = t.ms[i];
            if (launches) launches[i] = t.launches[i];
        }
        if (reset) t.reset();
    });
}

int fmm_plan_destroy(fmb_plan_t plan) {
    return guarded([&] { delete plan; });
}

}  // extern "C"
