// Shape derivatives of one wavenumber's point sum, and the self-triangle
// blocks of a given geometry: the two device parts of the gradient of a
// functional with respect to the mesh (Sec. 4, eq. 4.2 differentiated through
// the discretised system of eqs. 2.8 and 2.12).
//
// For fixed densities (a, b) and adjoint weights lam the point sum's bilinear form
//   B = sum_{alpha, beta: t(beta) != t(alpha)} w_beta [ grad'g . c + g e ],
//   u = conj(lam_alpha), c = (u . n_beta) a_beta - (u . a_beta) n_beta - (n_beta . a_beta) u,
//   e = u . b_beta,
// with d = s_beta - s_alpha, R = |d|, g = e^{ikR}/(4 pi R) (eq. 2.4), grad'g = f d,
// f = (ikR - 1) g / R^2, f'(R)/R = (3 - 3ikR + (ikR)^2) g / R^4, has
//   dB/ds_beta  = sum_alpha w_beta [ f c + ((f'/R)(d . c) + f e) d ],  dB/ds_alpha = -(the same, over beta)
//   dB/dn_beta  = sum_alpha w_beta f [ (d . a_beta) u - (u . a_beta) d - (d . u) a_beta ]
//   dB/dw_beta  = sum_alpha [ f (d . c) + g e ].
// Two direct O(n^2) FP64 passes, one thread per output node and the other side
// staged through LDS in tiles: every node as a target (its share of dB/ds), and
// every node as a source (dB/ds, dB/dn, dB/dw).  The other side is split into
// chunks (grid.y) so that a launch holds enough wavefronts to hide the latency
// of the per-pair sincos and exp; each chunk writes partial sums, which a last
// pass adds in chunk order (the result does not depend on scheduling).
#include <algorithm>

#include "plan.h"

namespace fmb {

namespace {

constexpr int SP_TILE = 128;
constexpr int SP_WAVES = 8192;       // wavefronts a launch aims at (about 8 per SIMD)
constexpr int SP_MAX_CHUNKS = 64;

struct SrcTile {
    double pos[SP_TILE][3];
    double nrm[SP_TILE][3];
    double w[SP_TILE];
    int32_t tri[SP_TILE];
    cx<double> a[SP_TILE][3], b[SP_TILE][3];
};

struct TgtTile {
    double pos[SP_TILE][3];
    int32_t tri[SP_TILE];
    cx<double> u[SP_TILE][3];
};

// g, f and f'/R of the pair at distance R (R > 0)
__device__ inline void pair_radial(double R, double k_re, double k_im, cx<double> &g, cx<double> &f, cx<double> &fp) {
    const double iR = 1.0 / R;
    double sn, cs;
    sincos(k_re * R, &sn, &cs);
    g = (0.07957747154594766788 * iR * exp(-k_im * R)) * mk(cs, sn);
    const cx<double> ikR = mk(-k_im * R, k_re * R);
    const double iR2 = iR * iR;
    f = iR2 * ((ikR - mk(1.0, 0.0)) * g);
    fp = (iR2 * iR2) * ((mk(3.0, 0.0) - 3.0 * ikR + ikR * ikR) * g);
}

// every node as a target: ds[alpha] = -sum_beta w_beta [ f c + ((f'/R)(d . c) + f e) d ]
__global__ void __launch_bounds__(SP_TILE) k_shape_tgt(const double *__restrict__ pts, const double *__restrict__ nrm,
                                                       const double *__restrict__ wts, const int32_t *__restrict__ tri,
                                                       const cx<double> *__restrict__ lam,
                                                       const cx<double> *__restrict__ a,
                                                       const cx<double> *__restrict__ b, int64_t n, int64_t chunk,
                                                       double k_re, double k_im, cx<double> *__restrict__ ds) {
    __shared__ SrcTile S;
    const int64_t al = blockIdx.x * (int64_t)SP_TILE + threadIdx.x;
    const int64_t lo = blockIdx.y * chunk, hi = min(n, lo + chunk);
    const bool active = al < n;
    double p[3] = {0, 0, 0};
    cx<double> u[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
    int32_t ta = -1;
    if (active) {
        for (int q = 0; q < 3; ++q) {
            p[q] = pts[3 * al + q];
            u[q] = conj(lam[3 * al + q]);
        }
        ta = tri[al];
    }
    cx<double> acc[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
    for (int64_t base = lo; base < hi; base += SP_TILE) {
        const int cnt = (int)min((int64_t)SP_TILE, hi - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const int j = threadIdx.x;
            const int64_t i = base + j;
            for (int q = 0; q < 3; ++q) {
                S.pos[j][q] = pts[3 * i + q];
                S.nrm[j][q] = nrm[3 * i + q];
                S.a[j][q] = a[3 * i + q];
                S.b[j][q] = b[3 * i + q];
            }
            S.w[j] = wts[i];
            S.tri[j] = tri[i];
        }
        __syncthreads();
        if (!active) continue;
        for (int j = 0; j < cnt; ++j) {
            if (S.tri[j] == ta) continue;
            const double d[3] = {S.pos[j][0] - p[0], S.pos[j][1] - p[1], S.pos[j][2] - p[2]};
            const double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (R2 <= 0.0) continue;
            cx<double> g, f, fp;
            pair_radial(sqrt(R2), k_re, k_im, g, f, fp);
            const double *nb = S.nrm[j];
            const cx<double> *ab = S.a[j], *bb = S.b[j];
            const cx<double> un = nb[0] * u[0] + nb[1] * u[1] + nb[2] * u[2];
            const cx<double> ua = u[0] * ab[0] + u[1] * ab[1] + u[2] * ab[2];
            const cx<double> na = nb[0] * ab[0] + nb[1] * ab[1] + nb[2] * ab[2];
            const cx<double> e = u[0] * bb[0] + u[1] * bb[1] + u[2] * bb[2];
            cx<double> c[3];
            for (int q = 0; q < 3; ++q) c[q] = un * ab[q] - nb[q] * ua - na * u[q];
            const cx<double> dc = d[0] * c[0] + d[1] * c[1] + d[2] * c[2];
            const cx<double> rad = fp * dc + f * e;
            const double w = S.w[j];
            for (int q = 0; q < 3; ++q) acc[q] -= w * (f * c[q] + d[q] * rad);
        }
    }
    if (!active) return;
    cx<double> *o = ds + 3 * ((int64_t)blockIdx.y * n + al);
    for (int q = 0; q < 3; ++q) o[q] = acc[q];
}

// every node as a source: ds[beta] += w_beta sum_alpha [ f c + ((f'/R)(d . c) + f e) d ],
// dn[beta] = w_beta sum_alpha f [ (d . a) u - (u . a) d - (d . u) a ], dw[beta] = sum_alpha [ f (d . c) + g e ]
__global__ void __launch_bounds__(SP_TILE) k_shape_src(const double *__restrict__ pts, const double *__restrict__ nrm,
                                                       const double *__restrict__ wts, const int32_t *__restrict__ tri,
                                                       const cx<double> *__restrict__ lam,
                                                       const cx<double> *__restrict__ a,
                                                       const cx<double> *__restrict__ b, int64_t n, int64_t chunk,
                                                       double k_re, double k_im, cx<double> *__restrict__ ds,
                                                       cx<double> *__restrict__ dn, cx<double> *__restrict__ dw) {
    __shared__ TgtTile S;
    const int64_t be = blockIdx.x * (int64_t)SP_TILE + threadIdx.x;
    const int64_t lo = blockIdx.y * chunk, hi = min(n, lo + chunk);
    const bool active = be < n;
    double p[3] = {0, 0, 0}, nb[3] = {0, 0, 0}, w = 0.0;
    cx<double> ab[3], bb[3];
    for (int q = 0; q < 3; ++q) ab[q] = bb[q] = mk(0.0, 0.0);
    int32_t tb = -1;
    if (active) {
        for (int q = 0; q < 3; ++q) {
            p[q] = pts[3 * be + q];
            nb[q] = nrm[3 * be + q];
            ab[q] = a[3 * be + q];
            bb[q] = b[3 * be + q];
        }
        w = wts[be];
        tb = tri[be];
    }
    const cx<double> na = nb[0] * ab[0] + nb[1] * ab[1] + nb[2] * ab[2];
    cx<double> as[3], an[3], aw = mk(0.0, 0.0);
    for (int q = 0; q < 3; ++q) as[q] = an[q] = mk(0.0, 0.0);
    for (int64_t base = lo; base < hi; base += SP_TILE) {
        const int cnt = (int)min((int64_t)SP_TILE, hi - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const int j = threadIdx.x;
            const int64_t i = base + j;
            for (int q = 0; q < 3; ++q) {
                S.pos[j][q] = pts[3 * i + q];
                S.u[j][q] = conj(lam[3 * i + q]);
            }
            S.tri[j] = tri[i];
        }
        __syncthreads();
        if (!active) continue;
        for (int j = 0; j < cnt; ++j) {
            if (S.tri[j] == tb) continue;
            const double d[3] = {p[0] - S.pos[j][0], p[1] - S.pos[j][1], p[2] - S.pos[j][2]};
            const double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (R2 <= 0.0) continue;
            cx<double> g, f, fp;
            pair_radial(sqrt(R2), k_re, k_im, g, f, fp);
            const cx<double> *u = S.u[j];
            const cx<double> un = nb[0] * u[0] + nb[1] * u[1] + nb[2] * u[2];
            const cx<double> ua = u[0] * ab[0] + u[1] * ab[1] + u[2] * ab[2];
            const cx<double> e = u[0] * bb[0] + u[1] * bb[1] + u[2] * bb[2];
            const cx<double> da = d[0] * ab[0] + d[1] * ab[1] + d[2] * ab[2];
            const cx<double> du = d[0] * u[0] + d[1] * u[1] + d[2] * u[2];
            cx<double> c[3];
            for (int q = 0; q < 3; ++q) c[q] = un * ab[q] - nb[q] * ua - na * u[q];
            const cx<double> dc = d[0] * c[0] + d[1] * c[1] + d[2] * c[2];
            const cx<double> rad = fp * dc + f * e;
            for (int q = 0; q < 3; ++q) {
                as[q] += f * c[q] + d[q] * rad;
                an[q] += f * (da * u[q] - d[q] * ua - du * ab[q]);
            }
            aw += f * dc + g * e;
        }
    }
    if (!active) return;
    const int64_t e = (int64_t)blockIdx.y * n + be;
    for (int q = 0; q < 3; ++q) {
        ds[3 * e + q] = w * as[q];
        dn[3 * e + q] = w * an[q];
    }
    dw[e] = aw;
}

// the partial sums of the chunks, added in chunk order: ds from both passes, dn, dw
__global__ void k_shape_sum(const cx<double> *__restrict__ pt, const cx<double> *__restrict__ ps,
                            const cx<double> *__restrict__ pn, const cx<double> *__restrict__ pw, int64_t n,
                            int chunks, cx<double> *__restrict__ ds, cx<double> *__restrict__ dn,
                            cx<double> *__restrict__ dw) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    cx<double> s[3], t[3], u[3], v = mk(0.0, 0.0);
    for (int q = 0; q < 3; ++q) s[q] = t[q] = u[q] = mk(0.0, 0.0);
    for (int c = 0; c < chunks; ++c) {
        const int64_t e = (int64_t)c * n + i;
        for (int q = 0; q < 3; ++q) {
            s[q] += pt[3 * e + q];
            t[q] += ps[3 * e + q];
            u[q] += pn[3 * e + q];
        }
        v += pw[e];
    }
    for (int q = 0; q < 3; ++q) {
        ds[3 * i + q] = s[q] + t[q];
        dn[3 * i + q] = u[q];
    }
    dw[i] = v;
}

}  // namespace

}  // namespace fmb

using namespace fmb;

extern "C" {

int bem_shape_pairs(const double *points, const double *normals, const double *weights, const int32_t *point_tri,
                    int64_t n, double k_re, double k_im, const void *lam, const void *a, const void *b, void *ds,
                    void *dn, void *dw, void *stream) {
    return guarded([&] {
        FMB_REQUIRE(n >= 1, "n must be >= 1");
        FMB_REQUIRE(n <= (int64_t)INT32_MAX, "n must fit in int32");
        FMB_REQUIRE(points && normals && weights && point_tri && lam && a && b && ds && dn && dw,
                    "every pointer is required");
        FMB_REQUIRE(std::isfinite(k_re) && std::isfinite(k_im) && k_im >= 0.0, "k must be finite with k_im >= 0");
        const void *outs[3] = {ds, dn, dw};
        const void *ins[7] = {points, normals, weights, point_tri, lam, a, b};
        for (const void *o : outs)
            for (const void *i : ins) FMB_REQUIRE(o != i, "outputs must not alias inputs");
        FMB_REQUIRE(ds != dn && ds != dw && dn != dw, "ds, dn and dw must be distinct");
        hipStream_t s = (hipStream_t)stream;
        const int64_t tiles = (n + SP_TILE - 1) / SP_TILE;
        // chunks of whole tiles of the other side: about SP_WAVES wavefronts per launch
        int64_t want = (SP_WAVES + 2 * tiles - 1) / (2 * tiles);
        want = std::max<int64_t>(1, std::min<int64_t>({want, tiles, (int64_t)SP_MAX_CHUNKS}));
        const int64_t chunk = ((tiles + want - 1) / want) * SP_TILE;
        const int chunks = (int)((n + chunk - 1) / chunk);
        DevBuf part;
        part.alloc((size_t)chunks * n * 10 * sizeof(cx<double>));
        cx<double> *pt = part.as<cx<double>>(), *ps = pt + (size_t)chunks * n * 3, *pn = ps + (size_t)chunks * n * 3,
                   *pw = pn + (size_t)chunks * n * 3;
        const dim3 grid((unsigned)tiles, (unsigned)chunks);
        k_shape_tgt<<<grid, SP_TILE, 0, s>>>(points, normals, weights, point_tri, (const cx<double> *)lam,
                                             (const cx<double> *)a, (const cx<double> *)b, n, chunk, k_re, k_im, pt);
        FMB_LAUNCH_CHECK();
        k_shape_src<<<grid, SP_TILE, 0, s>>>(points, normals, weights, point_tri, (const cx<double> *)lam,
                                             (const cx<double> *)a, (const cx<double> *)b, n, chunk, k_re, k_im, ps,
                                             pn, pw);
        FMB_LAUNCH_CHECK();
        k_shape_sum<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(pt, ps, pn, pw, n, chunks, (cx<double> *)ds,
                                                                (cx<double> *)dn, (cx<double> *)dw);
        FMB_LAUNCH_CHECK();
        FMB_CHECK_HIP(hipStreamSynchronize(s));    // the partial sums are freed on return
    });
}

int bem_self_blocks(const double *points, const double *normals, const int32_t *point_tri, const double *tri_vertices,
                    int64_t n, int64_t ntri, int32_t mode, double k_re, double k_im, void *dv, void *dg,
                    void *stream) {
    return guarded([&] {
        FMB_REQUIRE(points && normals && point_tri && tri_vertices && dv && dg, "every pointer is required");
        FMB_REQUIRE(n >= 1 && ntri >= 1 && n <= (int64_t)INT32_MAX, "need n >= 1 and ntri >= 1");
        FMB_REQUIRE(n % ntri == 0 && (n / ntri == 1 || n / ntri == 3),
                    "every triangle must hold 1 or 3 nodes (n / ntri in {1, 3})");
        FMB_REQUIRE(mode == FMB_CORR_MEAN || mode == FMB_CORR_LINEAR, "mode must be FMB_CORR_MEAN or FMB_CORR_LINEAR");
        FMB_REQUIRE(mode == FMB_CORR_MEAN || n / ntri == 3, "FMB_CORR_LINEAR needs 3 nodes per triangle");
        FMB_REQUIRE(std::isfinite(k_re) && std::isfinite(k_im) && k_im >= 0.0, "k must be finite with k_im >= 0");
        FMB_REQUIRE(dv != dg, "dv and dg must be distinct");
        for (int64_t i = 0; i < 3 * n; ++i) FMB_REQUIRE(std::isfinite(points[i]), "non-finite point");
        for (int64_t i = 0; i < n; ++i) {
            const double *v = normals + 3 * i;
            FMB_REQUIRE(std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]), "non-finite normal");
            FMB_REQUIRE(std::fabs(v[0] * v[0] + v[1] * v[1] + v[2] * v[2] - 1.0) <= 2e-6, "normals must be unit");
            FMB_REQUIRE(point_tri[i] >= 0 && point_tri[i] < ntri, "point_tri entry out of range");
        }
        for (int64_t i = 0; i < 9 * ntri; ++i) FMB_REQUIRE(std::isfinite(tri_vertices[i]), "non-finite vertex");
        hipStream_t s = (hipStream_t)stream;
        Plan P;
        P.n = n;
        P.ntri = ntri;
        P.tri_m = n / ntri;
        P.corr_mode = mode;
        P.k_re = k_re;
        P.k_im = k_im;
        DevBuf d_pts, d_nrm, d_tv;
        d_pts.alloc(3 * n * sizeof(double));
        d_nrm.alloc(3 * n * sizeof(double));
        d_tv.alloc(9 * ntri * sizeof(double));
        P.point_tri.alloc(n * sizeof(int32_t));
        FMB_CHECK_HIP(hipMemcpyAsync(d_pts.p, points, 3 * n * sizeof(double), hipMemcpyHostToDevice, s));
        FMB_CHECK_HIP(hipMemcpyAsync(d_nrm.p, normals, 3 * n * sizeof(double), hipMemcpyHostToDevice, s));
        FMB_CHECK_HIP(hipMemcpyAsync(d_tv.p, tri_vertices, 9 * ntri * sizeof(double), hipMemcpyHostToDevice, s));
        FMB_CHECK_HIP(hipMemcpyAsync(P.point_tri.p, point_tri, n * sizeof(int32_t), hipMemcpyHostToDevice, s));
        build_corrections(P, d_pts.as<double>(), d_nrm.as<double>(), d_tv.as<double>(), s);
        const size_t m = (size_t)P.tri_m;
        FMB_CHECK_HIP(hipMemcpyAsync(dv, P.corr_v.p, (size_t)n * m * 3 * sizeof(cx<double>), hipMemcpyDeviceToDevice, s));
        FMB_CHECK_HIP(hipMemcpyAsync(dg, P.corr_g.p, (size_t)n * m * sizeof(cx<double>), hipMemcpyDeviceToDevice, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
    });
}

}  // extern "C"
