// Translation operators of the upward and downward passes (eqs. 2.20-2.21),
// built in FP64 on the GPU.
//
// Expansions use R_n^m = j_n(k r) Y_n^m and S_n^m = h_n(k r) Y_n^m (eq. 2.16)
// with Y of eq. 2.15.  From the plane-wave form of the regular solutions,
// R_n^m(r) = (1/(4 pi i^n)) int exp(i k khat.r) Y_n^m(khat) dOmega, one gets the
// re-expansion of a basis function about a shifted centre,
//
//   F_n^m(r + t) = sum_{n',m'} T[n'm', nm](t) G_{n'}^{m'}(r),
//   T[n'm', nm](t) = sum_l 4 pi i^(n' + l - n) Gaunt(n,m; n',m'; l) X_l^{m-m'}(t),
//   Gaunt(n,m; n',m'; l) = int Y_n^m conj(Y_n'^m') conj(Y_l^(m-m')) dOmega,
//
// with (F, G, X) = (R, R, R) for R|R, (S, S, R) for S|S (|r| > |t|) and
// (S, R, S) for S|R (|r| < |t|).  A vector of expansion coefficients c
// (field = sum_nm c_nm F_n^m(. - centre)) re-expanded about a centre moved by
// -t becomes T(t) c.  The Gaunt integrals are exact Gauss-Legendre sums in
// cos(theta) (the phi integral only selects mu = m - m').
//
// Scaled coefficients.  To keep every coefficient near unit size in FP32 the
// library stores Mtilde_n = M_n / alpha_n(l) and Ltilde_n = L_n alpha_n(l) with
// alpha_n(l) = |j_n(i |k| rho_l)| (modified spherical Bessel i_n), rho_l the
// radius of a level-l box.  The operators built here include these factors.
#include "plan.h"

namespace fmb {

namespace {

constexpr int TPB = 256;

// Gauss-Legendre nodes/weights on [-1,1] by Newton iteration on P_Q.
__global__ void k_gauss_legendre(int Q, double *x, double *w) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (Q + 1) / 2) return;
    const double pi = 3.14159265358979323846;
    double z = cos(pi * (i + 0.75) / (Q + 0.5));
    double pp = 0.0;
    for (int it = 0; it < 100; ++it) {
        double p1 = 1.0, p2 = 0.0;
        for (int j = 1; j <= Q; ++j) {
            double p3 = p2;
            p2 = p1;
            p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        pp = Q * (z * p1 - p2) / (z * z - 1.0);
        double z1 = z;
        z = z1 - p1 / pp;
        if (fabs(z - z1) < 1e-15) {
            // one more step's derivative at the converged node
            p1 = 1.0;
            p2 = 0.0;
            for (int j = 1; j <= Q; ++j) {
                double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            pp = Q * (z * p1 - p2) / (z * z - 1.0);
            break;
        }
    }
    x[i] = -z;
    x[Q - 1 - i] = z;
    double wi = 2.0 / ((1.0 - z * z) * pp * pp);
    w[i] = wi;
    w[Q - 1 - i] = wi;
}

// Q_l^m(x) for l <= Lm, m <= l at the Q nodes: tab[node][l][m]
__global__ void k_qtab(const double *x, int Q, int Lm, double *tab) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Q) return;
    const double xi = x[i];
    const int S = Lm + 1;
    double *t = tab + (size_t)i * S * S;
    double qmm = 1.0 / sqrt(4.0 * 3.14159265358979323846);
    for (int m = 0; m <= Lm; ++m) {
        if (m > 0) qmm *= sqrt((2.0 * m + 1.0) / (2.0 * m));
        t[m * S + m] = qmm;
        if (m + 1 <= Lm) t[(m + 1) * S + m] = sqrt(2.0 * m + 3.0) * xi * qmm;
        for (int l = m + 2; l <= Lm; ++l) {
            double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            double b = sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
            t[l * S + m] = a * (xi * t[(l - 1) * S + m] - b * t[(l - 2) * S + m]);
        }
    }
}

__device__ inline void nm_of(int idx, int &n, int &m) {
    n = (int)sqrt((double)idx);
    while (n * n > idx) --n;
    while ((n + 1) * (n + 1) <= idx) ++n;
    m = idx - n * n - n;
}

// gaunt[src][dst][l]
__global__ void k_gaunt(int p, int Q, const double *w, const double *x, const double *tab, double *gaunt) {
    const int P2 = p * p;
    const int Lm = 2 * p - 2;
    const int S = Lm + 1;
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)P2 * P2) return;
    int src = (int)(e / P2), dst = (int)(e % P2);
    int n, m, n2, m2;
    nm_of(src, n, m);
    nm_of(dst, n2, m2);
    int mu = m - m2;
    double *g = gaunt + e * (Lm + 1);
    for (int l = 0; l <= Lm; ++l) g[l] = 0.0;
    int am = abs(m), am2 = abs(m2), amu = abs(mu);
    int pw2 = am + am2 + amu;   // even
    for (int l = abs(n - n2); l <= n + n2; l += 2) {
        if (amu > l) continue;
        double s = 0.0;
        for (int i = 0; i < Q; ++i) {
            const double *t = tab + (size_t)i * S * S;
            double sn2 = 1.0 - x[i] * x[i];
            double sp = 1.0;
            for (int q = 0; q < pw2 / 2; ++q) sp *= sn2;
            s += w[i] * t[n * S + am] * t[n2 * S + am2] * t[l * S + amu] * sp;
        }
        g[l] = 2.0 * 3.14159265358979323846 * s;
    }
}

// alpha_n(l) = |j_n(i x)|, x = |k| rho_l
__global__ void k_alpha(double kabs, double ext, int depth, int p, double *alpha) {
    int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l > depth) return;
    double rho = 0.5 * sqrt(3.0) * ext / (double)(1 << l);
    cx<double> jb[64];
    sph_bessel_j(mk(0.0, kabs * rho), p, jb);
    for (int n = 0; n < p; ++n) {
        double a = sqrt(abs2(jb[n]));
        alpha[l * p + n] = a > 1e-300 ? a : 1e-300;
    }
}

struct OpDesc {
    double t[3];
    int kind;          // 0: X = R (regular), 1: X = S (singular)
    int out_slot;      // slot index in the output array
    int dst_level, src_level;
    int dst_inv, src_inv;   // 1: multiply by 1/alpha instead of alpha
};

template <typename TO>
__global__ void k_build_op(OpDesc const *__restrict__ descs, int p, double k_re, double k_im,
                           const double *__restrict__ gaunt, const double *__restrict__ alpha, TO *__restrict__ out) {
    const int P2 = p * p;
    const int Lm = 2 * p - 2;
    const int NL = (Lm + 1) * (Lm + 1);
    extern __shared__ double sh[];
    cx<double> *F = reinterpret_cast<cx<double> *>(sh);          // [NL]
    cx<double> *rad = F + NL;                                      // [Lm+1]
    __shared__ double sd[32], ss[32];
    const OpDesc d = descs[blockIdx.x];
    const double tr = sqrt(d.t[0] * d.t[0] + d.t[1] * d.t[1] + d.t[2] * d.t[2]);
    const cx<double> k = mk(k_re, k_im);
    if (threadIdx.x == 0) {
        cx<double> z = k * tr;
        if (d.kind == 0) sph_bessel_j(z, Lm, rad);
        else sph_hankel_h1(z, Lm, rad);
    }
    if (threadIdx.x < p) {
        int nn = threadIdx.x;
        double ad = alpha[d.dst_level * p + nn], as = alpha[d.src_level * p + nn];
        sd[nn] = d.dst_inv ? 1.0 / ad : ad;
        ss[nn] = d.src_inv ? 1.0 / as : as;
    }
    __syncthreads();
    // Y_l^mu(that) column by column: thread per m >= 0
    const double xc = tr > 0 ? d.t[2] / tr : 1.0;
    const cx<double> wv = tr > 0 ? mk(d.t[0] / tr, d.t[1] / tr) : mk(0.0, 0.0);
    for (int m = threadIdx.x; m <= Lm; m += blockDim.x) {
        // Q_m^m and w^m
        double qmm = 1.0 / sqrt(4.0 * 3.14159265358979323846);
        cx<double> wm = mk(1.0, 0.0);
        for (int i = 1; i <= m; ++i) {
            qmm *= sqrt((2.0 * i + 1.0) / (2.0 * i));
            wm = wm * wv;
        }
        double sgn = (m & 1) ? -1.0 : 1.0;
        double q2 = 0.0, q1 = qmm;
        for (int l = m; l <= Lm; ++l) {
            double q;
            if (l == m) q = qmm;
            else if (l == m + 1) q = sqrt(2.0 * m + 3.0) * xc * qmm;
            else {
                double a = sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
                double b = sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
                q = a * (xc * q1 - b * q2);
            }
            if (l > m) {
                q2 = q1;
                q1 = q;
            }
            cx<double> Y = (sgn * q) * wm;
            F[l * l + l + m] = rad[l] * Y;
            if (m > 0) F[l * l + l - m] = rad[l] * conj(Y);
        }
    }
    __syncthreads();
    // real embedding: 2x2 block [[re, -im], [im, re]] at (2 dst, 2 src)
    const int KR = 2 * P2;
    TO *T = out + (size_t)d.out_slot * KR * KR;
    for (int e = threadIdx.x; e < P2 * P2; e += blockDim.x) {
        int dst = e / P2, src = e % P2;
        int n, m, n2, m2;
        nm_of(src, n, m);
        nm_of(dst, n2, m2);
        int mu = m - m2;
        const double *g = gaunt + ((size_t)src * P2 + dst) * (Lm + 1);
        cx<double> acc = mk(0.0, 0.0);
        for (int l = abs(n - n2); l <= n + n2; l += 2) {
            if (abs(mu) > l) continue;
            int ph = ((n2 + l - n) % 4 + 4) % 4;   // i^ph
            cx<double> ip = ph == 0 ? mk(1.0, 0.0) : ph == 1 ? mk(0.0, 1.0) : ph == 2 ? mk(-1.0, 0.0) : mk(0.0, -1.0);
            acc += (4.0 * 3.14159265358979323846 * g[l]) * (ip * F[l * l + l + mu]);
        }
        acc = (sd[n2] * ss[n]) * acc;
        T[(size_t)(2 * dst) * KR + 2 * src] = (TO)acc.re;
        T[(size_t)(2 * dst) * KR + 2 * src + 1] = (TO)(-acc.im);
        T[(size_t)(2 * dst + 1) * KR + 2 * src] = (TO)acc.im;
        T[(size_t)(2 * dst + 1) * KR + 2 * src + 1] = (TO)acc.re;
    }
}

}  // namespace

// Recurrence constants for the basis kernels (P2M, L2P), N = order:
//   la[n][m] = sqrt((4n^2 - 1) / (n^2 - m^2)), lb[n][m] = sqrt(((n-1)^2 - m^2) / (4(n-1)^2 - 1))  (n >= m + 2),
//   qmm[m] = Q_m^m / (sin th)^m = (4 pi)^{-1/2} prod_{i <= m} sqrt((2i + 1) / 2i),  q1[m] = sqrt(2m + 3),
// then, per coefficient idx = n^2 + n + m (n < order) with mu = -m, the six
// coefficients and R-table indices of the gradient recurrences
//   d_z R_n^mu = k (-A R_{n+1}^mu + B R_{n-1}^mu)
//   d_+ R_n^mu = k s_u (-c R_{n+1}^{mu+1} + d R_{n-1}^{mu+1})    (s_u = sign of mu, +1 at 0)
//   d_- R_n^mu = k s_d (-e R_{n+1}^{mu-1} + f R_{n-1}^{mu-1})    (s_d = +1 for mu > 0, else -1)
// and the index of R_n^mu itself; terms outside 0 <= n <= N, |mu| <= n point
// at the zero entry (N+1)^2.
void build_basis_tables(Plan &P, hipStream_t s) {
    const int N = P.order, NN = (N + 1) * (N + 1), P2 = P.order * P.order;
    std::vector<double> t((size_t)2 * NN + 2 * (N + 1) + (size_t)6 * P2, 0.0);
    double *la = t.data(), *lb = la + NN, *qmm = lb + NN, *q1 = qmm + (N + 1), *gco = q1 + (N + 1);
    for (int m = 0; m <= N; ++m)
        for (int n = m + 2; n <= N; ++n) {
            la[n * (N + 1) + m] = std::sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
            lb[n * (N + 1) + m] = std::sqrt(((double)(n - 1) * (n - 1) - (double)m * m) / (4.0 * (n - 1) * (n - 1) - 1.0));
        }
    qmm[0] = 0.28209479177387814347;
    for (int m = 1; m <= N; ++m) qmm[m] = qmm[m - 1] * std::sqrt((2.0 * m + 1.0) / (2.0 * m));
    for (int m = 0; m <= N; ++m) q1[m] = std::sqrt(2.0 * m + 3.0);
    std::vector<int32_t> gix((size_t)7 * P2);
    auto at = [&](int n, int mu) { return (n < 0 || n > N || mu > n || mu < -n) ? NN : n * n + n + mu; };
    for (int idx = 0; idx < P2; ++idx) {
        int n = 0;
        while ((n + 1) * (n + 1) <= idx) ++n;
        const int mu = -(idx - n * n - n);
        const int am = mu < 0 ? -mu : mu;
        const double A = std::sqrt((double)(n + 1 - am) * (n + 1 + am) / ((2.0 * n + 1) * (2.0 * n + 3)));
        const double B = n > 0 ? std::sqrt((double)(n - am) * (n + am) / ((2.0 * n - 1) * (2.0 * n + 1))) : 0.0;
        const double c = -std::sqrt((double)(n + mu + 1) * (n + mu + 2) / ((2.0 * n + 1) * (2.0 * n + 3)));
        const double d = (n > 0 && (n - mu) * (n - mu - 1) > 0)
                             ? std::sqrt((double)(n - mu) * (n - mu - 1) / ((2.0 * n - 1) * (2.0 * n + 1)))
                             : 0.0;
        const double e = std::sqrt((double)(n - mu + 1) * (n - mu + 2) / ((2.0 * n + 1) * (2.0 * n + 3)));
        const double f = (n > 0 && (n + mu) * (n + mu - 1) > 0)
                             ? -std::sqrt((double)(n + mu) * (n + mu - 1) / ((2.0 * n - 1) * (2.0 * n + 1)))
                             : 0.0;
        const double su = mu >= 0 ? 1.0 : -1.0, sd = mu > 0 ? 1.0 : -1.0;
        double *g = gco + (size_t)6 * idx;
        g[0] = -A;
        g[1] = B;
        g[2] = -su * c;
        g[3] = su * d;
        g[4] = -sd * e;
        g[5] = sd * f;
        int32_t *ix = gix.data() + (size_t)7 * idx;
        ix[0] = at(n + 1, mu);
        ix[1] = at(n - 1, mu);
        ix[2] = at(n + 1, mu + 1);
        ix[3] = at(n - 1, mu + 1);
        ix[4] = at(n + 1, mu - 1);
        ix[5] = at(n - 1, mu - 1);
        ix[6] = at(n, mu);
    }
    if (P.precision == FMB_FP64) {
        P.btab.alloc(t.size() * sizeof(double));
        FMB_CHECK_HIP(hipMemcpyAsync(P.btab.p, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice, s));
    } else {
        std::vector<float> tf(t.begin(), t.end());
        P.btab.alloc(tf.size() * sizeof(float));
        FMB_CHECK_HIP(hipMemcpyAsync(P.btab.p, tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice, s));
    }
    P.bgix.alloc(gix.size() * sizeof(int32_t));
    FMB_CHECK_HIP(hipMemcpyAsync(P.bgix.p, gix.data(), gix.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    FMB_CHECK_HIP(hipStreamSynchronize(s));
}

void build_operators(Plan &P, hipStream_t s) {
    const int p = P.order, P2 = p * p, L = P.depth;
    const int Lm = 2 * p - 2;
    const int Q = 2 * p + 2;
    const size_t esz = P.precision == FMB_FP64 ? sizeof(double) : sizeof(float);
    DevBuf gx, gw, tab, gaunt;
    gx.alloc(Q * sizeof(double));
    gw.alloc(Q * sizeof(double));
    tab.alloc((size_t)Q * (Lm + 1) * (Lm + 1) * sizeof(double));
    gaunt.alloc((size_t)P2 * P2 * (Lm + 1) * sizeof(double));
    k_gauss_legendre<<<1, 64, 0, s>>>(Q, gx.as<double>(), gw.as<double>());
    k_qtab<<<1, 64, 0, s>>>(gx.as<double>(), Q, Lm, tab.as<double>());
    k_gaunt<<<(unsigned)(((int64_t)P2 * P2 + TPB - 1) / TPB), TPB, 0, s>>>(p, Q, gw.as<double>(), gx.as<double>(),
                                                                              tab.as<double>(), gaunt.as<double>());
    FMB_LAUNCH_CHECK();
    P.inv_alpha.alloc((size_t)(L + 1) * p * sizeof(double));
    DevBuf alpha;
    alpha.alloc((size_t)(L + 1) * p * sizeof(double));
    const double kabs = sqrt(P.k_re * P.k_re + P.k_im * P.k_im);
    k_alpha<<<1, 64, 0, s>>>(kabs, P.ext, L, p, alpha.as<double>());
    FMB_LAUNCH_CHECK();
    {
        std::vector<double> ha((L + 1) * p), hi((L + 1) * p);
        FMB_CHECK_HIP(hipMemcpyAsync(ha.data(), alpha.p, ha.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
        for (size_t i = 0; i < ha.size(); ++i) hi[i] = 1.0 / ha[i];
        FMB_CHECK_HIP(hipMemcpyAsync(P.inv_alpha.p, hi.data(), hi.size() * sizeof(double), hipMemcpyHostToDevice, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
    }
    build_basis_tables(P, s);
    const size_t shmem = ((size_t)(Lm + 1) * (Lm + 1) + (Lm + 1)) * sizeof(cx<double>);
    auto launch = [&](std::vector<OpDesc> &ds, DevBuf &outbuf, int nslots) {
        outbuf.alloc((size_t)nslots * P2 * P2 * 4 * esz);
        if (ds.empty()) return;
        DevBuf dd;
        dd.alloc(ds.size() * sizeof(OpDesc));
        FMB_CHECK_HIP(hipMemcpyAsync(dd.p, ds.data(), ds.size() * sizeof(OpDesc), hipMemcpyHostToDevice, s));
        if (P.precision == FMB_FP64)
            k_build_op<double><<<(unsigned)ds.size(), TPB, shmem, s>>>(dd.as<OpDesc>(), p, P.k_re, P.k_im,
                                                                         gaunt.as<double>(), alpha.as<double>(),
                                                                         outbuf.as<double>());
        else
            k_build_op<float><<<(unsigned)ds.size(), TPB, shmem, s>>>(dd.as<OpDesc>(), p, P.k_re, P.k_im,
                                                                        gaunt.as<double>(), alpha.as<double>(),
                                                                        outbuf.as<float>());
        FMB_LAUNCH_CHECK();
        FMB_CHECK_HIP(hipStreamSynchronize(s));
    };
    // levels below far_lmin keep no far field (lossy cutoff): no operators there
    for (int l = std::max(2, P.far_lmin); l <= L; ++l) {
        Level &V = P.lv[l];
        const double h = P.ext / (double)(1 << l);
        // S|R for every far-field offset that occurs at this level
        std::vector<OpDesc> ds;
        for (int o = 0; o < N_M2L_OPS; ++o) {
            if (V.op_start[o + 1] == V.op_start[o]) continue;
            int dx = o / 49 - 3, dy = (o / 7) % 7 - 3, dz = o % 7 - 3;
            OpDesc d{};
            // offset = source coords - target coords; t = X_t - X_s
            d.t[0] = -dx * h;
            d.t[1] = -dy * h;
            d.t[2] = -dz * h;
            d.kind = 1;
            d.out_slot = o;
            d.dst_level = l;
            d.src_level = l;
            ds.push_back(d);
        }
        launch(ds, V.m2l, N_M2L_OPS);
        // S|S from the children (level l+1) into this level: t = X_parent - X_child
        if (l < L) {
            std::vector<OpDesc> dm;
            const double hc = P.ext / (double)(1 << (l + 1));
            for (int o = 0; o < 8; ++o) {
                OpDesc d{};
                for (int a = 0; a < 3; ++a) d.t[a] = -(((o >> a) & 1) - 0.5) * hc;
                d.kind = 0;
                d.out_slot = o;
                d.dst_level = l;
                d.src_level = l + 1;
                d.dst_inv = 1;
                dm.push_back(d);
            }
            launch(dm, V.m2m, 8);
        }
        // R|R from the parent (level l-1) into this level: t = X_child - X_parent
        if (l >= 3 && l > P.far_lmin) {
            std::vector<OpDesc> dl;
            for (int o = 0; o < 8; ++o) {
                OpDesc d{};
                for (int a = 0; a < 3; ++a) d.t[a] = (((o >> a) & 1) - 0.5) * h;
                d.kind = 0;
                d.out_slot = o;
                d.dst_level = l;
                d.src_level = l - 1;
                d.src_inv = 1;
                dl.push_back(d);
            }
            launch(dl, V.l2l, 8);
        }
    }
}

}  // namespace fmb
