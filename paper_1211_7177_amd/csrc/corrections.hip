// Self-triangle correction blocks (Appendix B), FP64 on the GPU.
//
// For a node O of triangle T (normal n) the element integrals are taken in
// polar coordinates about O (Fig. B.1).  Edge e has the foot D_e of the
// perpendicular from O, h_e = |OD_e|, i_e = OD_e/h_e, j_e = n x i_e, and is
// swept by phi in [phi1_e, phi2_e] with rho_m = h_e / cos(phi),
// rho^ = cos(phi) i_e + sin(phi) j_e.  With z = i k rho_m:
//
//   int_T g dA          = (1/4pi) sum_e int (e^z - 1)/(i k) dphi
//   CPV int_T grad'g dA = -(1/4pi) CPV int_T r/r^3 dA
//                         + (1/4pi) sum_e int rho^ H(z) dphi,
//       CPV int_T r/r^3 dA = sum_e i_e ln[tan(pi/4 - th2/2) / tan(pi/4 + th1/2)]   (eq. B.9),
//       H(z) = sum_{n>=2} (n-1) z^n / (n n!)   (the regular remainder; eqs. B.4-B.5
//              keep only its leading term), summed for |z| < 4 and taken in closed
//              form through the exponential integral E1 otherwise
//   int_T g (s'-O) dA      = (1/4pi) sum_e int rho^ [(1 - z) e^z - 1]/k^2 dphi
//   int_T grad'g (s'-O)^T  = (1/4pi) sum_e int rho^ rho^T [rho_m e^z - 2 (e^z - 1)/(i k)] dphi
//
// The two first moments give the linear-interpolation blocks: node beta of T
// with Lagrange function L_beta gets
//   dG = L_beta(O) G + grad L_beta . int g (s'-O) dA,
//   dV = L_beta(O) V + [int grad'g (s'-O)^T dA] grad L_beta,
// and grad L_j = n x (P_{j+2} - P_{j+1}) / (n . ((P_1 - P_0) x (P_2 - P_0))) for
// the triangle's nodes P_0..P_2.  The angular integrals use a fixed 64-node
// Gauss-Legendre rule per edge.
#include "plan.h"

namespace fmb {

namespace {

constexpr int TPB = 128;
constexpr int NQ = 64;

__constant__ double c_glx[NQ];
__constant__ double c_glw[NQ];

struct V3 {
    double x, y, z;
};
__device__ inline V3 v3(const double *p) { return V3{p[0], p[1], p[2]}; }
__device__ inline V3 operator-(V3 a, V3 b) { return V3{a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 operator+(V3 a, V3 b) { return V3{a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline V3 operator*(double s, V3 a) { return V3{s * a.x, s * a.y, s * a.z}; }
__device__ inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 cross(V3 a, V3 b) { return V3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }

__device__ inline cx<double> H_series(cx<double> z) {
    // sum_{n>=2} (n-1) z^n / (n n!)
    cx<double> term = (0.5) * (z * z);    // z^2/2!
    cx<double> out = mk(0.0, 0.0);
    for (int n = 2; n < 80; ++n) {
        out += ((double)(n - 1) / (double)n) * term;
        term = term * z * (1.0 / (double)(n + 1));
        if (abs2(term) < 1e-36 * abs2(out) && n > 4) break;
    }
    return out;
}

// E1(w), the exponential integral, for Re w >= 0 and |w| >= 2: the continued
// fraction E1(w) = e^{-w} / (w + 1 - 1^2/(w + 3 - 2^2/(w + 5 - ...))), evaluated
// forward by the modified Lentz method.
__device__ inline cx<double> E1_cf(cx<double> w) {
    cx<double> f = w + mk(1.0, 0.0), C = f, D = mk(0.0, 0.0);
    for (int j = 1; j < 2000; ++j) {
        const double a = -(double)j * (double)j;
        const cx<double> b = w + mk(2.0 * j + 1.0, 0.0);
        D = cdiv(mk(1.0, 0.0), b + a * D);
        C = b + a * cdiv(mk(1.0, 0.0), C);
        const cx<double> d = C * D;
        f = f * d;
        if (abs2(d - mk(1.0, 0.0)) < 1e-32) break;
    }
    return cdiv(cexp_(-w), f);
}

__device__ inline cx<double> H_closed(cx<double> z) {
    // H(z) = int_0^z [(u - 1) e^u + 1]/u du = e^z - 1 - F(z), F(z) = int_0^z (e^u - 1)/u du,
    // and F(z) = -E1(-z) - ln(-z) - gamma on the principal branches (Re(-z) = Im k rho >= 0)
    const cx<double> w = -z;
    const cx<double> lw = mk(0.5 * log(abs2(w)), atan2(w.im, w.re));
    return cexp_(z) - mk(1.0 - 0.57721566490153286061, 0.0) + E1_cf(w) + lw;
}

__global__ void k_tri_nodes_fill(const int32_t *__restrict__ point_tri, int64_t n, int m, int32_t *__restrict__ cnt,
                                 int32_t *__restrict__ nodes, int32_t *__restrict__ bad) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t t = point_tri[i];
    int32_t slot = atomicAdd(&cnt[t], 1);
    if (slot < m) nodes[(int64_t)t * m + slot] = (int32_t)i;
    else atomicOr(bad, 1);
}

__global__ void k_tri_nodes_sort(int32_t *__restrict__ nodes, const int32_t *__restrict__ cnt, int64_t ntri, int m,
                                 int32_t *__restrict__ bad) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= ntri) return;
    if (cnt[t] != m) {
        atomicOr(bad, 1);
        return;
    }
    int32_t *a = nodes + t * m;
    for (int i = 1; i < m; ++i)
        for (int j = i; j > 0 && a[j - 1] > a[j]; --j) {
            int32_t x = a[j];
            a[j] = a[j - 1];
            a[j - 1] = x;
        }
}

__global__ void k_corr_build(const double *__restrict__ pts, const double *__restrict__ nrm,
                             const int32_t *__restrict__ point_tri, const double *__restrict__ tri,
                             const int32_t *__restrict__ tri_nodes, int64_t n, int m, int mode, double k_re,
                             double k_im, cx<double> *__restrict__ cv, cx<double> *__restrict__ cg) {
    int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= n) return;
    const double pi = 3.14159265358979323846;
    const cx<double> k = mk(k_re, k_im);
    const cx<double> ik = mk(-k_im, k_re);
    const V3 O = v3(pts + 3 * a);
    const V3 nn = v3(nrm + 3 * a);
    const int32_t t = point_tri[a];
    const double *tv = tri + 9 * (int64_t)t;
    cx<double> G = mk(0.0, 0.0), Gv[3], V[3], W[3][3];
    for (int i = 0; i < 3; ++i) {
        Gv[i] = mk(0.0, 0.0);
        V[i] = mk(0.0, 0.0);
        for (int j = 0; j < 3; ++j) W[i][j] = mk(0.0, 0.0);
    }
    double stat[3] = {0.0, 0.0, 0.0};
    const bool need_moments = (mode == FMB_CORR_LINEAR && m == 3);
    for (int e = 0; e < 3; ++e) {
        V3 A = v3(tv + 3 * e), B = v3(tv + 3 * ((e + 1) % 3));
        V3 tvec = B - A;
        double len = sqrt(dot(tvec, tvec));
        V3 tu = (1.0 / len) * tvec;
        V3 D = A + dot(O - A, tu) * tu;
        V3 OD = D - O;
        double h = sqrt(dot(OD, OD));
        V3 ie = (1.0 / h) * OD;
        V3 je = cross(nn, ie);
        double p1 = atan2(dot(A - D, je), h);
        double p2 = atan2(dot(B - D, je), h);
        // eq. B.9 term of this edge: ln tan(pi/4 - p2/2) - ln tan(pi/4 - p1/2)
        double lr = log(tan(0.25 * pi - 0.5 * p2)) - log(tan(0.25 * pi - 0.5 * p1));
        stat[0] += lr * ie.x;
        stat[1] += lr * ie.y;
        stat[2] += lr * ie.z;
        const double half = 0.5 * (p2 - p1);
        for (int q = 0; q < NQ; ++q) {
            double phi = half * (c_glx[q] + 1.0) + p1;
            double jac = half * c_glw[q];
            double cph = cos(phi), sph = sin(phi);
            double rho = h / cph;
            V3 rh = cph * ie + sph * je;
            cx<double> z = mk(-k_im * rho, k_re * rho);
            double az = sqrt(abs2(z));
            cx<double> E = cexp_(z);
            cx<double> gi;
            if (az < 1e-4) gi = rho * (mk(1.0, 0.0) + 0.5 * z + (1.0 / 6.0) * (z * z));
            else gi = cdiv(E - mk(1.0, 0.0), ik);
            G += jac * gi;
            cx<double> Hv = az < 4.0 ? H_series(z) : H_closed(z);
            V[0] += (jac * rh.x) * Hv;
            V[1] += (jac * rh.y) * Hv;
            V[2] += (jac * rh.z) * Hv;
            if (need_moments) {
                cx<double> f1;
                if (az < 0.1) {
                    // rho^2 sum_{n>=2} (n-1) z^(n-2) / n!
                    cx<double> ser = mk(0.0, 0.0), term = mk(0.5, 0.0);
                    for (int nn2 = 2; nn2 < 18; ++nn2) {
                        ser += (double)(nn2 - 1) * term;
                        term = term * z * (1.0 / (double)(nn2 + 1));
                    }
                    f1 = (rho * rho) * ser;
                } else {
                    f1 = cdiv((mk(1.0, 0.0) - z) * E - mk(1.0, 0.0), k * k);
                }
                cx<double> f2 = rho * E - 2.0 * cdiv(E - mk(1.0, 0.0), ik);
                double r3[3] = {rh.x, rh.y, rh.z};
                for (int i = 0; i < 3; ++i) {
                    Gv[i] += (jac * r3[i]) * f1;
                    for (int j = 0; j < 3; ++j) W[i][j] += (jac * r3[i] * r3[j]) * f2;
                }
            }
        }
    }
    const double s4 = 1.0 / (4.0 * pi);
    G = s4 * G;
    for (int i = 0; i < 3; ++i) {
        V[i] = s4 * (V[i] - mk(i == 0 ? stat[0] : (i == 1 ? stat[1] : stat[2]), 0.0));
        Gv[i] = s4 * Gv[i];
        for (int j = 0; j < 3; ++j) W[i][j] = s4 * W[i][j];
    }
    const int32_t *nodes = tri_nodes + (int64_t)t * m;
    for (int j = 0; j < m; ++j) {
        cx<double> dV[3], dG;
        if (!need_moments) {
            double f = 1.0 / (double)m;
            for (int i = 0; i < 3; ++i) dV[i] = f * V[i];
            dG = f * G;
        } else {
            V3 P0 = v3(pts + 3 * (int64_t)nodes[0]), P1 = v3(pts + 3 * (int64_t)nodes[1]),
               P2 = v3(pts + 3 * (int64_t)nodes[2]);
            double two_area = dot(nn, cross(P1 - P0, P2 - P0));
            V3 Pa = j == 0 ? P1 : (j == 1 ? P2 : P0);   // P_{j+1}
            V3 Pb = j == 0 ? P2 : (j == 1 ? P0 : P1);   // P_{j+2}
            V3 gL = (1.0 / two_area) * cross(nn, Pb - Pa);
            double g3[3] = {gL.x, gL.y, gL.z};
            const bool self = nodes[j] == (int32_t)a;
            dG = mk(0.0, 0.0);
            for (int i = 0; i < 3; ++i) dG += g3[i] * Gv[i];
            if (self) dG += G;
            for (int i = 0; i < 3; ++i) {
                dV[i] = mk(0.0, 0.0);
                for (int q = 0; q < 3; ++q) dV[i] += g3[q] * W[i][q];
                if (self) dV[i] += V[i];
            }
        }
        for (int i = 0; i < 3; ++i) cv[(a * m + j) * 3 + i] = dV[i];
        cg[a * m + j] = dG;
    }
}

}  // namespace

// The matvec's last step: y[alpha] = ys[iperm[alpha]] (the FMM result, Morton
// order, gathered back to user order) plus the self-triangle terms of alpha,
//   sum_j [ n_b (dV.a_b) - (n_b.dV) a_b - dV (n_b.a_b) + dG b_b ],  b = tri_nodes[t(alpha)][j],
// in one pass over the nodes.
template <typename T>
__global__ void k_scatter_corr(const cx<T> *__restrict__ ys, const int32_t *__restrict__ iperm,
                               const cx<T> *__restrict__ a, const cx<T> *__restrict__ b, cx<T> *__restrict__ y,
                               const double *__restrict__ unrm, const int32_t *__restrict__ point_tri,
                               const int32_t *__restrict__ tri_nodes, const cx<double> *__restrict__ cv,
                               const cx<double> *__restrict__ cg, int64_t n, int m, int nrhs) {
    int64_t al = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (al >= n) return;
    const int32_t t = point_tri[al];
    const int64_t im = iperm[al];
    for (int r = 0; r < nrhs; ++r) {
        const int64_t off = (int64_t)r * n;
        cx<double> acc[3];
        for (int i = 0; i < 3; ++i) {
            const cx<T> v = ys[(off + im) * 3 + i];
            acc[i] = mk((double)v.re, (double)v.im);
        }
        for (int j = 0; j < m; ++j) {
            const int32_t be = tri_nodes[(int64_t)t * m + j];
            const double nb[3] = {unrm[3 * (int64_t)be], unrm[3 * (int64_t)be + 1], unrm[3 * (int64_t)be + 2]};
            cx<double> A[3], B[3], dV[3];
            for (int i = 0; i < 3; ++i) {
                cx<T> av = a[(off + be) * 3 + i], bv = b[(off + be) * 3 + i];
                A[i] = mk((double)av.re, (double)av.im);
                B[i] = mk((double)bv.re, (double)bv.im);
                dV[i] = cv[(al * m + j) * 3 + i];
            }
            const cx<double> dG = cg[al * m + j];
            cx<double> Va = dV[0] * A[0] + dV[1] * A[1] + dV[2] * A[2];
            cx<double> nV = nb[0] * dV[0] + nb[1] * dV[1] + nb[2] * dV[2];
            cx<double> na = nb[0] * A[0] + nb[1] * A[1] + nb[2] * A[2];
            for (int i = 0; i < 3; ++i) acc[i] += nb[i] * Va - nV * A[i] - dV[i] * na + dG * B[i];
        }
        for (int i = 0; i < 3; ++i) y[(off + al) * 3 + i] = mk((T)acc[i].re, (T)acc[i].im);
    }
}

void scatter_with_corrections(Plan &P, const void *ys, const void *a, const void *b, void *y, int nrhs,
                              hipStream_t s) {
    const unsigned g = (unsigned)((P.n + 255) / 256);
    if (P.precision == FMB_FP64)
        k_scatter_corr<double><<<g, 256, 0, s>>>((const cx<double> *)ys, P.iperm.as<int32_t>(),
                                                  (const cx<double> *)a, (const cx<double> *)b, (cx<double> *)y,
                                                  P.unrm.as<double>(), P.point_tri.as<int32_t>(),
                                                  P.tri_nodes.as<int32_t>(), P.corr_v.as<cx<double>>(),
                                                  P.corr_g.as<cx<double>>(), P.n, (int)P.tri_m, nrhs);
    else
        k_scatter_corr<float><<<g, 256, 0, s>>>((const cx<float> *)ys, P.iperm.as<int32_t>(), (const cx<float> *)a,
                                                 (const cx<float> *)b, (cx<float> *)y, P.unrm.as<double>(),
                                                 P.point_tri.as<int32_t>(), P.tri_nodes.as<int32_t>(),
                                                 P.corr_v.as<cx<double>>(), P.corr_g.as<cx<double>>(), P.n,
                                                 (int)P.tri_m, nrhs);
    FMB_LAUNCH_CHECK();
}

void build_corrections(Plan &P, const double *d_pts, const double *d_nrm, const double *d_tri, hipStream_t s) {
    const int64_t n = P.n;
    const int m = (int)P.tri_m;
    // Gauss-Legendre nodes: computed once on the host by Newton's method, kept in constant memory
    {
        std::vector<double> x(NQ), w(NQ);
        const double pi = 3.14159265358979323846;
        for (int i = 0; i < (NQ + 1) / 2; ++i) {
            double z = cos(pi * (i + 0.75) / (NQ + 0.5)), pp = 0.0;
            for (int it = 0; it < 100; ++it) {
                double p1 = 1.0, p2 = 0.0;
                for (int j = 1; j <= NQ; ++j) {
                    double p3 = p2;
                    p2 = p1;
                    p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
                }
                pp = NQ * (z * p1 - p2) / (z * z - 1.0);
                double z1 = z;
                z = z1 - p1 / pp;
                if (fabs(z - z1) < 1e-15) break;
            }
            x[i] = -z;
            x[NQ - 1 - i] = z;
            w[i] = w[NQ - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
        }
        FMB_CHECK_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_glx), x.data(), NQ * sizeof(double), 0,
                                             hipMemcpyHostToDevice, s));
        FMB_CHECK_HIP(hipMemcpyToSymbolAsync(HIP_SYMBOL(c_glw), w.data(), NQ * sizeof(double), 0,
                                             hipMemcpyHostToDevice, s));
    }
    P.tri_nodes.alloc((size_t)P.ntri * m * sizeof(int32_t));
    DevBuf cnt, bad;
    cnt.alloc(P.ntri * sizeof(int32_t));
    bad.alloc(sizeof(int32_t));
    FMB_CHECK_HIP(hipMemsetAsync(cnt.p, 0, P.ntri * sizeof(int32_t), s));
    FMB_CHECK_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    k_tri_nodes_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(P.point_tri.as<int32_t>(), n, m, cnt.as<int32_t>(),
                                                                 P.tri_nodes.as<int32_t>(), bad.as<int32_t>());
    k_tri_nodes_sort<<<(unsigned)((P.ntri + 255) / 256), 256, 0, s>>>(P.tri_nodes.as<int32_t>(), cnt.as<int32_t>(),
                                                                      P.ntri, m, bad.as<int32_t>());
    FMB_LAUNCH_CHECK();
    int32_t hb = 0;
    FMB_CHECK_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FMB_CHECK_HIP(hipStreamSynchronize(s));
    FMB_REQUIRE(hb == 0, "every triangle must hold exactly n/ntri nodes (1 or 3)");
    P.corr_v.alloc((size_t)n * m * 3 * sizeof(cx<double>));
    P.corr_g.alloc((size_t)n * m * sizeof(cx<double>));
    k_corr_build<<<(unsigned)((n + TPB - 1) / TPB), TPB, 0, s>>>(
        d_pts, d_nrm, P.point_tri.as<int32_t>(), d_tri, P.tri_nodes.as<int32_t>(), n, m, P.corr_mode, P.k_re, P.k_im,
        P.corr_v.as<cx<double>>(), P.corr_g.as<cx<double>>());
    FMB_LAUNCH_CHECK();
    FMB_CHECK_HIP(hipStreamSynchronize(s));
}

}  // namespace fmb
