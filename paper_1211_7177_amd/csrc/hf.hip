// Far field with a truncation order per level (plans built with order <= 0):
// the S|S, S|R and R|R translations of eqs. 2.20-2.21 by rotation, coaxial
// shift and rotation back, each target accumulating its own sources in a fixed
// order.
//
// A translation by t = (new centre - old centre) of a coefficient vector c
// (field = sum_nm c_nm F_n^m(x - old centre), F = R or S of eq. 2.16, Y of
// eq. 2.15) splits into three steps.  With theta, phi the angles of t and W^n
// the degree-n matrix of a rotation by theta about y,
//     Y_n^m(R_y(theta) x) = sum_m' W^n_{m m'}(theta) Y_n^m'(x),
//   1. c'_n^m'  = sum_m W^n_{m m'}(theta) e^{i m phi} c_n^m        (t turned onto +z)
//   2. c''_n'^m = sum_n C^m_{n' n}(|t|) c'_n^m                      (shift along +z)
//   3. d_n^m'   = e^{-i m' phi} sum_m W^n_{m' m}(theta) c''_n^m     (turned back; W orthogonal)
// W^n_{m m'} = s_m s_m' d^n_{m' m}(theta) with Wigner's d (s_m = (-1)^m for
// m > 0, else 1: eq. 2.15's phase), built by the three-term recurrence in the
// degree from the single-term value at n = max(|m|, |m'|).  The coaxial
// coefficients (F_n^m(r + |t| z) = sum_n' C^m_{n'n} G_n'^m(r)) start from
// C^0_{n'0} = (-1)^n' sqrt(2n'+1) f_n'(k|t|) (f = h_n for S|R, j_n for S|S and
// R|R) and follow from the derivative rules of the basis,
//   d_z F_n^m = k (a_n^m F_{n-1}^m - b_n^m F_{n+1}^m),
//   (d_x + i d_y) F_n^m = k (e_n^m F_{n+1}^{m+1} + f_n^m F_{n-1}^{m+1})  (m >= 0),
// applied to both sides of the shifted expansion: one recurrence advances the
// source degree n, the other raises |m|.  Work per translation is O(p^3)
// instead of the O(p^4) of a dense operator, and the tables are small enough
// for orders in the hundreds (the coarse levels of electrically large bodies,
// where k d reaches 10^2: truncation below eq. 2.17 needs p ~ k d).
//
// Scaled coefficients: Mtilde_n = M_n / alpha_n(l), Ltilde_n = L_n alpha_n(l) with
// alpha_n(l) = 1 / max(1, x |h_n(x)|), x = |k| rho_l (rho_l the level's box
// radius); the tables carry the alpha factors so that stored coefficients and
// table entries stay near unit size in FP32 at every order.
#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <thread>
#include <tuple>

#include "plan.h"

namespace fmb {

namespace {

using cd = std::complex<double>;

constexpr int HTPB = 256;
constexpr size_t HF_LDS_MAX = 64 * 1024;

// ------------------------------------------------------------ host functions

// j_n(z), n = 0..N (Miller's downward ratio recurrence, then j_0 = sin z / z)
void host_sph_j(cd z, int N, std::vector<cd> &out) {
    out.assign(N + 1, cd(0.0, 0.0));
    const double az = std::abs(z);
    if (az < 1e-300) {
        out[0] = 1.0;
        return;
    }
    const int start = N + 32 + (int)(1.5 * az);
    cd r = 0.0;
    std::vector<cd> ratio(N + 1);
    for (int n = start; n >= 1; --n) {
        r = z / (double(2 * n + 1) - z * r);
        if (n <= N) ratio[n] = r;
    }
    out[0] = az < 1e-3 ? 1.0 - z * z / 6.0 + z * z * z * z / 120.0 : std::sin(z) / z;
    for (int n = 1; n <= N; ++n) out[n] = out[n - 1] * ratio[n];
}

// h_n^(1)(z), n = 0..N (upward recurrence)
void host_sph_h(cd z, int N, std::vector<cd> &out) {
    out.assign(N + 1, cd(0.0, 0.0));
    const cd i(0.0, 1.0);
    const cd e = std::exp(i * z);
    out[0] = -i * e / z;
    if (N >= 1) out[1] = -e * (z + i) / (z * z);
    for (int n = 1; n < N; ++n) out[n + 1] = double(2 * n + 1) / z * out[n] - out[n - 1];
}

// alpha_n = 1 / max(1, x |h_n(x)|), n < p
std::vector<double> hf_alpha(double x, int p) {
    std::vector<double> a(p, 1.0);
    if (x <= 0.0) return a;
    std::vector<cd> h;
    host_sph_h(cd(x, 0.0), p, h);
    for (int n = 0; n < p; ++n) {
        const double v = x * std::abs(h[n]);
        a[n] = (std::isfinite(v) && v > 1.0) ? 1.0 / v : (std::isfinite(v) ? 1.0 : 1e-300);
        if (a[n] < 1e-300) a[n] = 1e-300;
    }
    return a;
}

// sum_{n < p} (2n+1)^2
inline int64_t wsize(int p) { return (int64_t)p * (2 * p - 1) * (2 * p + 1) / 3; }

// W[wsize(n) + (m+n)(2n+1) + (m'+n)] = s_m s_m' d^n_{m' m}(beta), n < p
void rotation_table(int p, double beta, double *W) {
    const double cb = std::cos(beta);
    const double ch = std::cos(0.5 * beta), sh = std::sin(0.5 * beta);
    const double lch = std::log(std::fabs(ch)), lsh = std::log(std::fabs(sh));
    auto s = [](int m) { return (m > 0 && (m & 1)) ? -1.0 : 1.0; };
    for (int mp = -(p - 1); mp <= p - 1; ++mp)
        for (int m = -(p - 1); m <= p - 1; ++m) {
            const int j0 = std::max(std::abs(m), std::abs(mp));
            // Wigner's sum has one term at j = j0: s = max(0, m - m')
            const int sv = std::max(0, m - mp);
            const double lg = 0.5 * (std::lgamma(j0 + mp + 1.0) + std::lgamma(j0 - mp + 1.0) +
                                     std::lgamma(j0 + m + 1.0) + std::lgamma(j0 - m + 1.0)) -
                              std::lgamma(j0 + m - sv + 1.0) - std::lgamma(sv + 1.0) -
                              std::lgamma(mp - m + sv + 1.0) - std::lgamma(j0 - mp - sv + 1.0);
            const int pc = 2 * j0 + m - mp - 2 * sv, ps = mp - m + 2 * sv;
            double d1;
            if ((pc > 0 && ch == 0.0) || (ps > 0 && sh == 0.0)) {
                d1 = 0.0;
            } else {
                const double v = lg + (pc > 0 ? pc * lch : 0.0) + (ps > 0 ? ps * lsh : 0.0);
                double sg = ((mp - m + sv) & 1) ? -1.0 : 1.0;
                if (pc > 0 && ch < 0.0 && (pc & 1)) sg = -sg;
                if (ps > 0 && sh < 0.0 && (ps & 1)) sg = -sg;
                d1 = sg * std::exp(v);
            }
            double d2 = 0.0;
            for (int j = j0; j < p; ++j) {
                double d;
                if (j == j0) {
                    d = d1;
                } else {
                    const double c1 = j * (2.0 * j - 1.0) / std::sqrt(((double)j * j - (double)m * m) * ((double)j * j - (double)mp * mp));
                    double t = (cb - (j > 1 ? (double)m * mp / ((double)j * (j - 1)) : 0.0)) * d1;
                    if (j - 1 > j0)
                        t -= std::sqrt(((j - 1.0) * (j - 1.0) - (double)m * m) * ((j - 1.0) * (j - 1.0) - (double)mp * mp)) /
                             ((j - 1.0) * (2.0 * j - 1.0)) * d2;
                    d = c1 * t;
                    d2 = d1;
                    d1 = d;
                }
                // W^j_{m, m'} = s_m s_m' d^j_{m', m}
                W[wsize(j) + (int64_t)(m + j) * (2 * j + 1) + (mp + j)] = s(m) * s(mp) * d;
            }
        }
}

// sum_{m < min(pd, ps)} (pd - m)(ps - m)
inline int64_t csize(int pd, int ps) {
    int64_t s = 0;
    for (int m = 0; m < std::min(pd, ps); ++m) s += (int64_t)(pd - m) * (ps - m);
    return s;
}

enum { CX_SR = 0, CX_SS = 1, CX_RR = 2 };

// coaxial coefficients C^m_{n'n}(t) along +z for n' < pd, n < ps, times the scale
// factors of the stored coefficients; block m at offset sum_{j<m}(pd-j)(ps-j),
// entry (n-m)(pd-m) + (n'-m) (consecutive output degrees n' adjacent)
// For S|S and R|R (regular translation function) the degree recurrence loses
// accuracy above the diagonal when k|t| is small (each step cancels terms a
// factor (k|t|)^2 larger than the result); there only the part n' >= n is
// recurred and the rest follows from the symmetry C^m_{n n'} = (-1)^(n+n') C^m_{n' n}
// of the regular re-expansion.  S|R keeps the full recurrence (its entries grow
// along it).
void coax_table(int kind, cd k, double t, int pd, int ps, const std::vector<double> &ad,
                const std::vector<double> &as, cd *out) {
    const bool sym = kind != CX_SR;
    const int pr = sym ? std::max(pd, ps) : pd;   // rows and columns recurred
    const int pc = sym ? std::max(pd, ps) : ps;
    const int N = pr + pc + 1;
    std::vector<cd> f;
    if (kind == CX_SR) host_sph_h(k * t, N, f);
    else host_sph_j(k * t, N, f);
    auto a_ = [](int n, int m) { return n > m ? std::sqrt((double)(n - m) * (n + m) / ((2.0 * n - 1) * (2.0 * n + 1))) : 0.0; };
    auto b_ = [](int n, int m) { return std::sqrt((n + 1.0 - m) * (n + 1.0 + m) / ((2.0 * n + 1) * (2.0 * n + 3))); };
    auto e_ = [](int n, int m) { return std::sqrt((n + m + 1.0) * (n + m + 2.0) / ((2.0 * n + 1) * (2.0 * n + 3))); };
    auto f_ = [](int n, int m) {
        return (n > 0 && n - m - 1 > 0) ? std::sqrt((double)(n - m) * (n - m - 1) / ((2.0 * n - 1) * (2.0 * n + 1))) : 0.0;
    };
    const int W = pc + 1;
    std::vector<cd> C((size_t)(N + 2) * W), prev(N + 2), cur(N + 2);
    auto at = [&](int q, int n) -> cd & { return C[(size_t)q * W + n]; };
    int64_t off = 0;
    for (int m = 0; m < std::min(pd, ps); ++m) {
        std::fill(C.begin(), C.end(), cd(0.0, 0.0));
        const int Nm = N - m;   // rows valid in column m
        if (m == 0) {
            for (int q = 0; q <= N; ++q) at(q, 0) = ((q & 1) ? -1.0 : 1.0) * std::sqrt(2.0 * q + 1.0) * f[q];
        } else {
            // C^m_{q, m} = [e^{m-1}_{q-1} C^{m-1}_{q-1, m-1} + f^{m-1}_{q+1} C^{m-1}_{q+1, m-1}] / e^{m-1}_{m-1}
            const double den = e_(m - 1, m - 1);
            for (int q = m; q <= Nm; ++q) at(q, m) = (e_(q - 1, m - 1) * prev[q - 1] + f_(q + 1, m - 1) * prev[q + 1]) / den;
        }
        for (int q = 0; q <= N + 1; ++q) prev[q] = q <= N ? at(q, m) : cd(0.0, 0.0);
        // C_{q, n+1} = [a_n C_{q, n-1} - a_{q+1} C_{q+1, n} + b_{q-1} C_{q-1, n}] / b_n
        for (int n = m; n < pc - 1; ++n) {
            const int qmax = Nm - (n - m) - 1;
            for (int q = sym ? n + 1 : m; q <= qmax; ++q) {
                cd v = -a_(q + 1, m) * at(q + 1, n);
                if (n - 1 >= m) v += a_(n, m) * at(q, n - 1);
                if (q - 1 >= m) v += b_(q - 1, m) * at(q - 1, n);
                at(q, n + 1) = v / b_(n, m);
            }
        }
        for (int q = m; q < pd; ++q)
            for (int n = m; n < ps; ++n) {
                double sc;
                if (kind == CX_SR) sc = ad[q] * as[n];
                else if (kind == CX_SS) sc = as[n] / ad[q];
                else sc = ad[q] / as[n];
                const cd v = (sym && q < n) ? (((q + n) & 1) ? -1.0 : 1.0) * at(n, q) : at(q, n);
                out[off + (int64_t)(n - m) * (pd - m) + (q - m)] = sc * v;
            }
        off += (int64_t)(pd - m) * (ps - m);
    }
}

template <typename T>
void upload_as(DevBuf &d, const std::vector<double> &v, hipStream_t s) {
    std::vector<T> h(v.begin(), v.end());
    d.alloc(std::max<size_t>(1, h.size()) * sizeof(T));
    if (!h.empty()) FMB_CHECK_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
    FMB_CHECK_HIP(hipStreamSynchronize(s));
}

template <typename T>
void upload_cx(DevBuf &d, const std::vector<cd> &v, hipStream_t s) {
    std::vector<cx<T>> h(v.size());
    for (size_t i = 0; i < v.size(); ++i) h[i] = mk((T)v[i].real(), (T)v[i].imag());
    d.alloc(std::max<size_t>(1, h.size()) * sizeof(cx<T>));
    if (!h.empty()) FMB_CHECK_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(cx<T>), hipMemcpyHostToDevice, s));
    FMB_CHECK_HIP(hipStreamSynchronize(s));
}

// run f(i) for i in [0, n) on up to 8 host threads
template <typename F>
void parallel_for(int n, F f) {
    const int nt = std::max(1, std::min(n, 8));
    std::vector<std::thread> th;
    for (int w = 0; w < nt; ++w)
        th.emplace_back([&, w] {
            for (int i = w; i < n; i += nt) f(i);
        });
    for (auto &x : th) x.join();
}

// ---------------------------------------------------------------- kernels

struct HfArgs {
    const void *W;       // rotation table of this translation's polar angle (covers max(ps, pd))
    const void *ph;      // e^{i m phi}, m = 0.. (covers max(ps, pd))
    const void *C;       // coaxial block table (pd x ps)
    int ps, pd;
};

// decode idx = n^2 + n + m
__device__ inline void hf_nm(int e, int &n, int &m) {
    n = (int)sqrtf((float)e);
    while (n * n > e) --n;
    while ((n + 1) * (n + 1) <= e) ++n;
    m = e - n * n - n;
}

// one translation of CH channel blocks (stride sstr between channels) into acc,
// with the two scratch vectors b1, b2 (each CH * max(ps, pd)^2)
template <typename T, int CH>
__device__ void hf_translate(const cx<T> *__restrict__ src, int64_t sstr, const T *__restrict__ W,
                             const cx<T> *__restrict__ ph, const cx<T> *__restrict__ C, int ps, int pd, cx<T> *b1,
                             cx<T> *b2, cx<T> *acc) {
    const int S2 = ps * ps, D2 = pd * pd;
    // 1: phases, source order ps
    for (int t = threadIdx.x; t < CH * S2; t += blockDim.x) {
        const int c = t / S2, e = t - c * S2;
        int n, m;
        hf_nm(e, n, m);
        const cx<T> f = m >= 0 ? ph[m] : conj(ph[-m]);
        b1[c * S2 + e] = f * src[c * sstr + e];
    }
    __syncthreads();
    // 2: rotation onto +z, c'_n^m' = sum_m W[n][m][m'] c_n^m
    for (int t = threadIdx.x; t < CH * S2; t += blockDim.x) {
        const int c = t / S2, e = t - c * S2;
        int n, mp;
        hf_nm(e, n, mp);
        const T *w = W + (int64_t)n * (2 * n - 1) * (2 * n + 1) / 3 + (mp + n);
        const cx<T> *x = b1 + c * S2 + n * n;
        cx<T> s = mk(T(0), T(0));
        for (int m = 0; m <= 2 * n; ++m) s += w[(int64_t)m * (2 * n + 1)] * x[m];
        b2[c * S2 + e] = s;
    }
    __syncthreads();
    // 3: coaxial shift, c''_n'^m = sum_n C^|m|_{n'n} c'_n^m, into order pd
    for (int t = threadIdx.x; t < CH * D2; t += blockDim.x) {
        const int c = t / D2, e = t - c * D2;
        int q, m;
        hf_nm(e, q, m);
        const int am = m < 0 ? -m : m;
        cx<T> s = mk(T(0), T(0));
        if (am < ps) {
            // block offset sum_{j < am} (pd - j)(ps - j)
            int64_t off = 0;
            for (int j = 0; j < am; ++j) off += (int64_t)(pd - j) * (ps - j);
            const cx<T> *col = C + off + (q - am);
            const cx<T> *x = b2 + c * S2;
            for (int n = am; n < ps; ++n) s += col[(int64_t)(n - am) * (pd - am)] * x[n * n + n + m];
        }
        b1[c * D2 + e] = s;
    }
    __syncthreads();
    // 4: rotation back, d_n^m' = e^{-i m' phi} sum_m W[n][m'][m] c''_n^m, accumulated;
    //    W[n][m'][m] = (-1)^(m-m') W[n][m][m'] (Wigner's d^n_{m m'} = (-1)^(m-m') d^n_{m' m}),
    //    read along m' so that neighbouring threads read neighbouring entries
    for (int t = threadIdx.x; t < CH * D2; t += blockDim.x) {
        const int c = t / D2, e = t - c * D2;
        int n, mp;
        hf_nm(e, n, mp);
        const T *w = W + (int64_t)n * (2 * n - 1) * (2 * n + 1) / 3 + (mp + n);
        const cx<T> *x = b1 + c * D2 + n * n;
        cx<T> s = mk(T(0), T(0));
        for (int m = 0; m <= 2 * n; ++m) {
            const T wm = w[(int64_t)m * (2 * n + 1)];
            s += (((m + mp + n) & 1) ? -wm : wm) * x[m];
        }
        const cx<T> f = mp >= 0 ? conj(ph[mp]) : ph[-mp];
        acc[c * D2 + e] += f * s;
    }
    __syncthreads();
}

template <typename T, int CH, bool GLB>
__device__ inline void hf_buffers(cx<T> *smem, cx<T> *gscr, int64_t P2m, int64_t D2, cx<T> *&b1, cx<T> *&b2,
                                  cx<T> *&acc) {
    cx<T> *base = smem;
    if (GLB) base = gscr + ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * (2 * CH * P2m + CH * D2);
    b1 = base;
    b2 = base + CH * P2m;
    acc = base + 2 * CH * P2m;
}

// M2L: target box b of the level sums, in list order, the S|R translations of its
// far-field sources; writes (overwrites) its local expansion.
template <typename T, int CH, bool GLB>
__global__ void __launch_bounds__(HTPB) k_hf_m2l(const int32_t *__restrict__ ff_ofs, const int32_t *__restrict__ ff_src,
                                                 const int32_t *__restrict__ ff_op, const int32_t *__restrict__ opi,
                                                 const T *__restrict__ W, int64_t wsz, const cx<T> *__restrict__ ph,
                                                 const cx<T> *__restrict__ C, int64_t csz, int p, int nrhs_max,
                                                 const cx<T> *__restrict__ M, cx<T> *__restrict__ Lout, cx<T> *gscr) {
    extern __shared__ __align__(16) unsigned char hf_smem[];
    const int b = blockIdx.x;
    const int col = blockIdx.y * CH;                 // first channel (r * 3 + c) of this block
    const int r = col / 3, c0 = col % 3;
    const int64_t P2 = (int64_t)p * p;
    cx<T> *b1, *b2, *acc;
    hf_buffers<T, CH, GLB>(reinterpret_cast<cx<T> *>(hf_smem), gscr, P2, P2, b1, b2, acc);
    for (int t = threadIdx.x; t < CH * P2; t += blockDim.x) acc[t] = mk(T(0), T(0));
    __syncthreads();
    const int e0 = ff_ofs[b], e1 = ff_ofs[b + 1];
    for (int e = e0; e < e1; ++e) {
        const int s = ff_src[e], o = ff_op[e];
        const int beta = opi[2 * o], dist = opi[2 * o + 1];
        hf_translate<T, CH>(M + (((int64_t)s * nrhs_max + r) * 3 + c0) * P2, P2, W + beta * wsz, ph + (int64_t)o * p,
                            C + dist * csz, p, p, b1, b2, acc);
    }
    cx<T> *out = Lout + (((int64_t)b * nrhs_max + r) * 3 + c0) * P2;
    for (int t = threadIdx.x; t < CH * P2; t += blockDim.x) out[t] = acc[t];
}

// M2M into parent box b (order pd) from its children (order ps, their own octant
// directions); writes the parent's multipole.
template <typename T, int CH, bool GLB>
__global__ void __launch_bounds__(HTPB) k_hf_m2m(const int32_t *__restrict__ child_start,
                                                 const int32_t *__restrict__ child_oct, const T *__restrict__ Wo,
                                                 int64_t wszo, const int32_t *__restrict__ beta_oct,
                                                 const cx<T> *__restrict__ pho, int pwo, const cx<T> *__restrict__ C,
                                                 int ps, int pd, int nrhs_max, const cx<T> *__restrict__ Mc,
                                                 cx<T> *__restrict__ Mp, cx<T> *gscr) {
    extern __shared__ __align__(16) unsigned char hf_smem[];
    const int b = blockIdx.x;
    const int col = blockIdx.y * CH;
    const int r = col / 3, c0 = col % 3;
    const int64_t S2 = (int64_t)ps * ps, D2 = (int64_t)pd * pd, P2m = S2 > D2 ? S2 : D2;
    cx<T> *b1, *b2, *acc;
    hf_buffers<T, CH, GLB>(reinterpret_cast<cx<T> *>(hf_smem), gscr, P2m, D2, b1, b2, acc);
    for (int t = threadIdx.x; t < CH * D2; t += blockDim.x) acc[t] = mk(T(0), T(0));
    __syncthreads();
    for (int ch = child_start[b]; ch < child_start[b + 1]; ++ch) {
        const int o = child_oct[ch];
        hf_translate<T, CH>(Mc + (((int64_t)ch * nrhs_max + r) * 3 + c0) * S2, S2, Wo + beta_oct[o] * wszo,
                            pho + (int64_t)o * pwo, C, (int)ps, (int)pd, b1, b2, acc);
    }
    cx<T> *out = Mp + (((int64_t)b * nrhs_max + r) * 3 + c0) * D2;
    for (int t = threadIdx.x; t < CH * D2; t += blockDim.x) out[t] = acc[t];
}

// L2L into child box b (order pd) from its parent (order ps): added to the
// child's local expansion (which holds its far-field sum).
template <typename T, int CH, bool GLB>
__global__ void __launch_bounds__(HTPB) k_hf_l2l(const int32_t *__restrict__ parent, const int32_t *__restrict__ oct,
                                                 const T *__restrict__ Wo, int64_t wszo,
                                                 const int32_t *__restrict__ beta_oct, const cx<T> *__restrict__ pho,
                                                 int pwo, const cx<T> *__restrict__ C, int ps, int pd, int nrhs_max,
                                                 const cx<T> *__restrict__ Lp, cx<T> *__restrict__ Lc, cx<T> *gscr) {
    extern __shared__ __align__(16) unsigned char hf_smem[];
    const int b = blockIdx.x;
    const int col = blockIdx.y * CH;
    const int r = col / 3, c0 = col % 3;
    const int64_t S2 = (int64_t)ps * ps, D2 = (int64_t)pd * pd, P2m = S2 > D2 ? S2 : D2;
    cx<T> *b1, *b2, *acc;
    hf_buffers<T, CH, GLB>(reinterpret_cast<cx<T> *>(hf_smem), gscr, P2m, D2, b1, b2, acc);
    cx<T> *out = Lc + (((int64_t)b * nrhs_max + r) * 3 + c0) * D2;
    for (int t = threadIdx.x; t < CH * D2; t += blockDim.x) acc[t] = out[t];
    __syncthreads();
    const int o = 8 + oct[b];
    hf_translate<T, CH>(Lp + (((int64_t)parent[b] * nrhs_max + r) * 3 + c0) * S2, S2, Wo + beta_oct[o] * wszo,
                        pho + (int64_t)o * pwo, C, (int)ps, (int)pd, b1, b2, acc);
    for (int t = threadIdx.x; t < CH * D2; t += blockDim.x) out[t] = acc[t];
}

template <typename T>
__global__ void k_hf_zero(cx<T> *__restrict__ x, int64_t m) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) x[i] = mk(T(0), T(0));
}

template <typename T>
size_t hf_lds(int ch, int64_t P2m, int64_t D2) { return (size_t)(2 * ch * P2m + ch * D2) * sizeof(cx<T>); }

// launch mode of a translation stage: 3 channels per block in LDS, 1 in LDS, or
// 1 with the scratch vectors in global memory (large orders)
template <typename T>
int hf_mode(int64_t P2m, int64_t D2) {
    if (hf_lds<T>(3, P2m, D2) <= HF_LDS_MAX) return 3;
    if (hf_lds<T>(1, P2m, D2) <= HF_LDS_MAX) return 1;
    return 0;
}

// ---------------------------------------------------------------- pipeline
// Large orders: each translation set in three launches that spread one
// translation over many blocks.  Pairs e carry a source box, a direction d
// (phase row, polar-angle class, distance class) and belong to a destination
// (CSR); the forward rotation and the coaxial shift go to per-pair scratch, and
// the back rotation walks each destination's pairs in order (deterministic).

__device__ inline int64_t hf_woff(int n) { return (int64_t)n * (2 * n - 1) * (2 * n + 1) / 3; }

template <typename T>
__device__ inline cx<T> hf_phase(const cx<T> *ph, int m) { return m >= 0 ? ph[m] : conj(ph[-m]); }

// position of item u within the |m|-blocks [m0, ...) of a coaxial shift to order
// pd, items ordered (|m|, sign, n'): returns |m|, m and n'
__device__ inline void hf_coax_item(int u, int m0, int pd, int &am, int &m, int &q) {
    am = m0;
    while (u >= (pd - am) * (am ? 2 : 1)) {
        u -= (pd - am) * (am ? 2 : 1);
        ++am;
    }
    const int len = pd - am;
    m = u < len ? am : -am;
    q = am + (u < len ? u : u - len);
}

// offset of block |m| = am in a coaxial table of orders (pd, ps): sum_{j < am} (pd - j)(ps - j)
__device__ inline int64_t hf_coff(int am, int pd, int ps) {
    return (int64_t)am * pd * ps - (int64_t)(pd + ps) * am * (am - 1) / 2 + (int64_t)(am - 1) * am * (2 * am - 1) / 6;
}

// X1[e][r][c][(n,m')] = sum_m W[n][m][m'] e^{i m phi} S[src][r][c][(n,m)], degrees [nck[z], nck[z+1]);
// the source's coefficients of those degrees, times the phases, are staged in LDS first; then one
// thread per coefficient, all three channels (one rotation-table read serves three)
template <typename T>
__global__ void __launch_bounds__(HTPB) k_hf_fwd(const int32_t *__restrict__ src_idx, const int32_t *__restrict__ dir,
                                                 int dir_add, const int32_t *__restrict__ dinfo,
                                                 const T *__restrict__ W, int64_t wsz, const cx<T> *__restrict__ ph,
                                                 int phs, const int32_t *__restrict__ nck, int ps, int nrhs_max,
                                                 int nrhs, const cx<T> *__restrict__ S, cx<T> *__restrict__ X1) {
    extern __shared__ __align__(16) unsigned char hf_smem[];
    cx<T> *xs = reinterpret_cast<cx<T> *>(hf_smem);
    const int e = blockIdx.x, r = blockIdx.y, z = blockIdx.z;
    const int n0 = nck[z], n1 = nck[z + 1];
    const int d = dir[e] + dir_add;
    const T *Wb = W + (int64_t)dinfo[2 * d] * wsz;
    const cx<T> *phd = ph + (int64_t)d * phs;
    const int64_t src = src_idx ? src_idx[e] : e;
    const int64_t P2 = (int64_t)ps * ps;
    const int base = n0 * n0, cnt = n1 * n1 - base;
    const cx<T> *S0 = S + (src * nrhs_max + r) * 3 * P2 + base;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
        int n, m;
        hf_nm(base + t, n, m);
        const cx<T> f = hf_phase(phd, m);
        xs[t] = f * S0[t];
        xs[cnt + t] = f * S0[P2 + t];
        xs[2 * cnt + t] = f * S0[2 * P2 + t];
    }
    __syncthreads();
    cx<T> *X0 = X1 + ((int64_t)e * nrhs + r) * 3 * P2;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
        const int ee = base + t;
        int n, mp;
        hf_nm(ee, n, mp);
        const T *w = Wb + hf_woff(n) + (mp + n);
        const cx<T> *x = xs + (n * n - base);
        cx<T> a0 = mk(T(0), T(0)), a1 = a0, a2 = a0;
        for (int m = 0; m <= 2 * n; ++m) {
            const T wm = w[(int64_t)m * (2 * n + 1)];
            a0 += wm * x[m];
            a1 += wm * x[cnt + m];
            a2 += wm * x[2 * cnt + m];
        }
        X0[ee] = a0;
        X0[P2 + ee] = a1;
        X0[2 * P2 + ee] = a2;
    }
}

// X2[e][r][c][(q,m)] = sum_n C^|m|_{q n} X1[e][r][c][(n,m)], |m| in [mck[z], mck[z+1]), q < pd;
// the inputs of those |m| are staged in LDS (item order (|m|, sign, n)); consecutive threads take
// consecutive q (adjacent table entries), all three channels
template <typename T>
__global__ void __launch_bounds__(HTPB) k_hf_coax(const int32_t *__restrict__ dir, int dir_add,
                                                  const int32_t *__restrict__ dinfo, const cx<T> *__restrict__ C,
                                                  int64_t csz, const int32_t *__restrict__ mck, int ps, int pd,
                                                  int nrhs, const cx<T> *__restrict__ X1, cx<T> *__restrict__ X2) {
    extern __shared__ __align__(16) unsigned char hf_smem[];
    cx<T> *xs = reinterpret_cast<cx<T> *>(hf_smem);
    const int e = blockIdx.x, r = blockIdx.y, z = blockIdx.z;
    const int m0 = mck[z], m1 = mck[z + 1];
    const int d = dir[e] + dir_add;
    const cx<T> *Cd = C + (int64_t)dinfo[2 * d + 1] * csz;
    const int64_t S2 = (int64_t)ps * ps, D2 = (int64_t)pd * pd;
    const int m1s = m1 < ps ? m1 : ps;
    int cin = 0, cnt = 0;
    for (int am = m0; am < m1; ++am) cnt += (pd - am) * (am ? 2 : 1);
    for (int am = m0; am < m1s; ++am) cin += (ps - am) * (am ? 2 : 1);
    const cx<T> *x = X1 + ((int64_t)e * nrhs + r) * 3 * S2;
    for (int t = threadIdx.x; t < cin; t += blockDim.x) {
        int am, m, n;
        hf_coax_item(t, m0, ps, am, m, n);
        const int i = n * n + n + m;
        xs[t] = x[i];
        xs[cin + t] = x[S2 + i];
        xs[2 * cin + t] = x[2 * S2 + i];
    }
    __syncthreads();
    cx<T> *y = X2 + ((int64_t)e * nrhs + r) * 3 * D2;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
        int am, m, q;
        hf_coax_item(t, m0, pd, am, m, q);
        cx<T> a0 = mk(T(0), T(0)), a1 = a0, a2 = a0;
        if (am < ps) {
            // this |m|'s staged inputs: items of the blocks before it, then the sign
            int at = 0;
            for (int j = m0; j < am; ++j) at += (ps - j) * (j ? 2 : 1);
            if (m < 0) at += ps - am;
            const cx<T> *col = Cd + hf_coff(am, pd, ps) + (q - am);
            const cx<T> *xi = xs + at;
            for (int n = am; n < ps; ++n) {
                const cx<T> cv = col[(int64_t)(n - am) * (pd - am)];
                a0 += cv * xi[n - am];
                a1 += cv * xi[cin + n - am];
                a2 += cv * xi[2 * cin + n - am];
            }
        }
        const int o = q * q + q + m;
        y[o] = a0;
        y[D2 + o] = a1;
        y[2 * D2 + o] = a2;
    }
}

// D[b][r][c][(n,m')] (=, or += with accumulate) sum over b's pairs e of
// e^{-i m' phi_e} sum_m W_e[n][m'][m] X2[e][r][c][(n,m)], degrees [nck[z], nck[z+1]);
// W[n][m'][m] = (-1)^(m-m') W[n][m][m'] (Wigner's d^n_{m m'} = (-1)^(m-m') d^n_{m' m}) is read along m';
// each pair's inputs of those degrees are staged in LDS
template <typename T>
__global__ void __launch_bounds__(HTPB) k_hf_back(const int32_t *__restrict__ dst_ofs, const int32_t *__restrict__ dir,
                                                  int dir_add, const int32_t *__restrict__ dinfo,
                                                  const T *__restrict__ W, int64_t wsz, const cx<T> *__restrict__ ph,
                                                  int phs, const int32_t *__restrict__ nck, int pd, int nrhs_max,
                                                  int nrhs, int accumulate, const cx<T> *__restrict__ X2,
                                                  cx<T> *__restrict__ D) {
    extern __shared__ __align__(16) unsigned char hf_smem[];
    cx<T> *xs = reinterpret_cast<cx<T> *>(hf_smem);
    const int b = blockIdx.x, r = blockIdx.y, z = blockIdx.z;
    const int n0 = nck[z], n1 = nck[z + 1];
    const int e0 = dst_ofs ? dst_ofs[b] : b, e1 = dst_ofs ? dst_ofs[b + 1] : b + 1;
    const int64_t D2 = (int64_t)pd * pd;
    const int base = n0 * n0, cnt = n1 * n1 - base;
    cx<T> *out = D + ((int64_t)b * nrhs_max + r) * 3 * D2;
    // each thread owns coefficients t = threadIdx.x + HTPB i; at most 4 per thread (chunks hold < 4 HTPB)
    cx<T> acc[4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = threadIdx.x + HTPB * i;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            acc[i][c] = (accumulate && t < cnt) ? out[c * D2 + base + t] : mk(T(0), T(0));
    }
    for (int e = e0; e < e1; ++e) {
        const int d = dir[e] + dir_add;
        const cx<T> *x = X2 + ((int64_t)e * nrhs + r) * 3 * D2 + base;
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
            xs[t] = x[t];
            xs[cnt + t] = x[D2 + t];
            xs[2 * cnt + t] = x[2 * D2 + t];
        }
        __syncthreads();
        const T *Wd = W + (int64_t)dinfo[2 * d] * wsz;
        const cx<T> *phd = ph + (int64_t)d * phs;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int t = threadIdx.x + HTPB * i;
            if (t < cnt) {
                int n, mp;
                hf_nm(base + t, n, mp);
                const T *w = Wd + hf_woff(n) + (mp + n);
                const cx<T> *xi = xs + (n * n - base);
                cx<T> s0 = mk(T(0), T(0)), s1 = s0, s2 = s0;
                for (int m = 0; m <= 2 * n; ++m) {
                    const T wm0 = w[(int64_t)m * (2 * n + 1)];
                    const T wm = ((m + mp + n) & 1) ? -wm0 : wm0;
                    s0 += wm * xi[m];
                    s1 += wm * xi[cnt + m];
                    s2 += wm * xi[2 * cnt + m];
                }
                const cx<T> f = hf_phase(phd, -mp);
                acc[i][0] += f * s0;
                acc[i][1] += f * s1;
                acc[i][2] += f * s2;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = threadIdx.x + HTPB * i;
        if (t < cnt) {
#pragma unroll
            for (int c = 0; c < 3; ++c) out[c * D2 + base + t] = acc[i][c];
        }
    }
}

// ------------------------------------------------------- small-order M2L
// Orders up to 20 (the fine levels, most boxes): one block per (target box,
// right-hand side), its four wavefronts translating four far-field sources at
// a time, each in its own LDS buffers.  A lane works on all three channels of
// a coefficient (one table read serves three).  Each lane keeps J of the
// target's coefficients in registers (t = lane + 64 j) and adds its
// wavefront's translations in list order; the four partial sums are added in
// wavefront order at the end (deterministic).
constexpr int HFW_WAVES = 4;

template <typename T, int J>
__global__ void __launch_bounds__(256) k_hf_m2l_w(const int32_t *__restrict__ ff_ofs, const int32_t *__restrict__ ff_src,
                                                  const int32_t *__restrict__ ff_op, const int32_t *__restrict__ opi,
                                                  const T *__restrict__ W, int64_t wsz, const cx<T> *__restrict__ ph,
                                                  const cx<T> *__restrict__ C, int64_t csz, int p, int nrhs_max,
                                                  const cx<T> *__restrict__ M, cx<T> *__restrict__ Lout) {
    extern __shared__ __align__(16) unsigned char hf_smem[];
    const int b = blockIdx.x, r = blockIdx.y;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int P2 = p * p, N3 = 3 * P2;
    // per wavefront two vectors of p^2 coefficients x 3 channels, channel-interleaved ([coefficient][3])
    cx<T> *A = reinterpret_cast<cx<T> *>(hf_smem) + (size_t)wv * 2 * N3;
    cx<T> *B = A + N3;
    // tab: (n, m + n) of coefficient t; tab2: (q, m + q) of the t-th coaxial item, ordered (|m|, sign, q)
    int32_t *tab = reinterpret_cast<int32_t *>(reinterpret_cast<cx<T> *>(hf_smem) + (size_t)HFW_WAVES * 2 * N3);
    int32_t *tab2 = tab + P2;
    for (int t = threadIdx.x; t < P2; t += blockDim.x) {
        int n, m;
        hf_nm(t, n, m);
        tab[t] = (n << 10) | (m + n);
        int am, q;
        hf_coax_item(t, 0, p, am, m, q);
        tab2[t] = (q << 10) | (m + q);
    }
    cx<T> acc[3 * J];
#pragma unroll
    for (int j = 0; j < 3 * J; ++j) acc[j] = mk(T(0), T(0));
    const int e0 = ff_ofs[b], cnt = ff_ofs[b + 1] - e0;
    __syncthreads();
    for (int base = 0; base < cnt; base += HFW_WAVES) {
        const bool act = base + wv < cnt;
        int s = 0, o = 0;
        if (act) {
            s = ff_src[e0 + base + wv];
            o = ff_op[e0 + base + wv];
        }
        const T *Wb = W + (int64_t)opi[2 * o] * wsz;
        const cx<T> *Cd = C + (int64_t)opi[2 * o + 1] * csz;
        const cx<T> *pho = ph + (int64_t)o * p;
        if (act) {
            // source coefficients times e^{i m phi}
            const cx<T> *src = M + ((int64_t)s * nrhs_max + r) * 3 * P2;
            for (int t = lane; t < P2; t += 64) {
                const int v = tab[t], n = v >> 10, m = (v & 1023) - n;
                const cx<T> f = hf_phase(pho, m);
                A[3 * t] = f * src[t];
                A[3 * t + 1] = f * src[P2 + t];
                A[3 * t + 2] = f * src[2 * P2 + t];
            }
        }
        __syncthreads();
        if (act) {
            // rotation onto +z: B_n^m' = sum_m W[n][m][m'] A_n^m
            for (int t = lane; t < P2; t += 64) {
                const int v = tab[t], n = v >> 10, mpn = v & 1023;
                const int st = 2 * n + 1;
                const T *w = Wb + hf_woff(n) + mpn;
                const cx<T> *x = A + 3 * n * n;
                cx<T> s0 = mk(T(0), T(0)), s1 = s0, s2 = s0;
#pragma unroll 4
                for (int m = 0; m < st; ++m) {
                    const T wm = w[m * st];
                    s0 += wm * x[3 * m];
                    s1 += wm * x[3 * m + 1];
                    s2 += wm * x[3 * m + 2];
                }
                B[3 * t] = s0;
                B[3 * t + 1] = s1;
                B[3 * t + 2] = s2;
            }
        }
        __syncthreads();
        if (act) {
            // coaxial shift: A_q^m = sum_n C^|m|_{q n} B_n^m
            for (int t = lane; t < P2; t += 64) {
                const int v = tab2[t], q = v >> 10, m = (v & 1023) - q;
                const int am = m < 0 ? -m : m;
                const int cs = p - am;
                const cx<T> *col = Cd + hf_coff(am, p, p) + (q - am);
                const cx<T> *x = B + 3 * (am * am + am + m);
                cx<T> s0 = mk(T(0), T(0)), s1 = s0, s2 = s0;
                // input n sits at 3 (n^2 + n + m); successive n are 3 (2n + 2) entries apart
                int off = 0;
#pragma unroll 2
                for (int n = am; n < p; ++n) {
                    const cx<T> cv = col[(n - am) * cs];
                    s0 += cv * x[off];
                    s1 += cv * x[off + 1];
                    s2 += cv * x[off + 2];
                    off += 6 * n + 6;
                }
                A[3 * (q * q + q + m)] = s0;
                A[3 * (q * q + q + m) + 1] = s1;
                A[3 * (q * q + q + m) + 2] = s2;
            }
        }
        __syncthreads();
        if (act) {
            // rotation back, d_n^m' = e^{-i m' phi} sum_m W[n][m'][m] c_n^m with W[n][m'][m] =
            // (-1)^(m-m') W[n][m][m'] read along m': the even-m and odd-m terms are summed apart and
            // combined with their signs at the end; added to this lane's coefficients
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int t = lane + 64 * j;
                if (t < P2) {
                    const int v = tab[t], n = v >> 10, mpn = v & 1023;
                    const int st = 2 * n + 1;
                    const T *w = Wb + hf_woff(n) + mpn;
                    const cx<T> *x = A + 3 * n * n;
                    cx<T> e0_ = mk(T(0), T(0)), e1_ = e0_, e2_ = e0_, o0 = e0_, o1 = e0_, o2 = e0_;
                    int m = 0;
#pragma unroll 2
                    for (; m + 1 < st; m += 2) {
                        const T we = w[m * st], wo = w[(m + 1) * st];
                        e0_ += we * x[3 * m];
                        e1_ += we * x[3 * m + 1];
                        e2_ += we * x[3 * m + 2];
                        o0 += wo * x[3 * m + 3];
                        o1 += wo * x[3 * m + 4];
                        o2 += wo * x[3 * m + 5];
                    }
                    {
                        const T we = w[m * st];           // m = 2n, even
                        e0_ += we * x[3 * m];
                        e1_ += we * x[3 * m + 1];
                        e2_ += we * x[3 * m + 2];
                    }
                    // (-1)^(m - m') = (-1)^(m + mpn) for m the index 0..2n
                    const T sg = (mpn & 1) ? T(-1) : T(1);
                    const cx<T> f = hf_phase(pho, n - mpn);
                    const cx<T> fs = sg * f;
                    acc[3 * j] += fs * (e0_ - o0);
                    acc[3 * j + 1] += fs * (e1_ - o1);
                    acc[3 * j + 2] += fs * (e2_ - o2);
                }
            }
        }
        __syncthreads();
    }
    // the four wavefronts' sums, added in wavefront order
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int t = lane + 64 * j;
        if (t < P2) {
            A[3 * t] = acc[3 * j];
            A[3 * t + 1] = acc[3 * j + 1];
            A[3 * t + 2] = acc[3 * j + 2];
        }
    }
    __syncthreads();
    cx<T> *out = Lout + ((int64_t)b * nrhs_max + r) * 3 * P2;
    const cx<T> *base0 = reinterpret_cast<cx<T> *>(hf_smem);
    for (int t = threadIdx.x; t < N3; t += blockDim.x) {
        const int c = t / P2, i = t - c * P2;
        cx<T> v = base0[3 * i + c];
        for (int w = 1; w < HFW_WAVES; ++w) v += base0[(size_t)w * 2 * N3 + 3 * i + c];
        out[t] = v;
    }
}

template <typename T>
size_t hfw_lds(int p) { return (size_t)HFW_WAVES * 2 * 3 * p * p * sizeof(cx<T>) + (size_t)2 * p * p * sizeof(int32_t); }

}  // namespace

// order needed at a level: the low-frequency floor for the tolerance, or the
// excess-bandwidth estimate k d + 1.8 d0^(2/3) (k d)^(1/3) (d the box diameter,
// d0 = digits) once boxes are many wavelengths across
int hf_order(double kabs, double side, double tol) {
    const double d0 = std::max(1.0, -std::log10(tol));
    const double kd = kabs * side * std::sqrt(3.0);
    const double pe = kd + 1.8 * std::pow(d0, 2.0 / 3.0) * std::cbrt(std::max(kd, 0.0));
    const double pf = 2.8 * d0;
    return (int)std::ceil(std::max(pe, pf));
}

// per-pair scratch of the pipeline: right-hand sides beyond what fits run in slices
constexpr size_t HF_PIPE_BYTES = (size_t)2 << 30;

// translation sets whose order exceeds this run as the three-launch pipeline;
// M2L at orders up to HFW_PMAX runs one source per wavefront
constexpr int HF_PIPE_P = 20;
// (its LDS, up to 157 KB per block for FP64 at order 20, fits the CU's 160 KB)
constexpr int HFW_PMAX = 20;
constexpr size_t HFW_LDS_MAX = 160 * 1024;

// chunk boundaries of the pipelined launches (one block per pair and chunk): about
// 256 coefficients per chunk and never more than HF_CHUNK_MAX, which is what the
// kernels' LDS staging and per-thread registers hold.  Degrees n < p:
constexpr int HF_CHUNK_MAX = 4 * HTPB;

static std::vector<int32_t> degree_chunks(int p, int &maxc) {
    std::vector<int32_t> v{0};
    int acc = 0;
    maxc = 0;
    for (int n = 0; n < p; ++n) {
        const int w = 2 * n + 1;
        if (acc > 0 && acc + w > HF_CHUNK_MAX) {
            v.push_back(n);
            maxc = std::max(maxc, acc);
            acc = 0;
        }
        acc += w;
        if (acc >= 256 || n == p - 1) {
            v.push_back(n + 1);
            maxc = std::max(maxc, acc);
            acc = 0;
        }
    }
    return v;
}

// |m| < pd for a coaxial shift from order ps to order pd: a block |m| holds
// (pd - |m|) outputs and (ps - |m|) inputs per sign, and both counts stay within a chunk
static std::vector<int32_t> m_chunks(int pd, int ps, int &maxc) {
    std::vector<int32_t> v{0};
    int acc = 0;
    maxc = 0;
    for (int am = 0; am < pd; ++am) {
        const int w = std::max(pd - am, std::max(ps - am, 0)) * (am ? 2 : 1);
        if (acc > 0 && acc + w > HF_CHUNK_MAX) {
            v.push_back(am);
            maxc = std::max(maxc, acc);
            acc = 0;
        }
        acc += w;
        if (acc >= 256 || am == pd - 1) {
            v.push_back(am + 1);
            maxc = std::max(maxc, acc);
            acc = 0;
        }
    }
    return v;
}

void build_hf(Plan &P, hipStream_t s) {
    const int L = P.depth;
    const int lmin = std::max(2, P.far_lmin);
    const cd k(P.k_re, P.k_im);
    const double kabs = std::abs(k);
    const bool f64 = P.precision == FMB_FP64;
    std::vector<std::vector<double>> alpha(L + 1);
    for (int l = 0; l <= L; ++l) {
        const double rho = 0.5 * std::sqrt(3.0) * P.ext / (double)(1 << l);
        alpha[l] = hf_alpha(kabs * rho, std::max(1, P.lv[l].p));
    }
    // 1/alpha at the leaf level for P2M / L2P (row layout [depth+1][order])
    {
        std::vector<double> ia((size_t)(L + 1) * P.order, 1.0);
        for (int n = 0; n < P.order; ++n) ia[(size_t)L * P.order + n] = 1.0 / alpha[L][n];
        upload_as<double>(P.inv_alpha, ia, s);
    }
    const double c1 = 1.0 / std::sqrt(3.0);
    for (int l = lmin; l <= L; ++l) {
        Level &V = P.lv[l];
        const int p = V.p;
        const double side = P.ext / (double)(1 << l);
        // --- far-field offsets used at this level: polar-angle and distance classes
        std::vector<int32_t> opi(2 * N_M2L_OPS, 0);
        std::map<std::pair<int, int>, int> bkey, dkey;
        std::vector<double> betas;
        std::vector<double> dists;
        std::vector<cd> ph((size_t)N_M2L_OPS * p, cd(0.0, 0.0));
        for (int o = 0; o < N_M2L_OPS; ++o) {
            if (V.op_start[o + 1] == V.op_start[o]) continue;
            const int dx = o / 49 - 3, dy = (o / 7) % 7 - 3, dz = o % 7 - 3;
            // offset = source - target box coordinates; t = X_t - X_s = -offset * side
            const double tx = -dx * side, ty = -dy * side, tz = -dz * side;
            const double T = std::sqrt(tx * tx + ty * ty + tz * tz);
            const std::pair<int, int> kb{-dz, dx * dx + dy * dy};
            if (!bkey.count(kb)) {
                bkey[kb] = (int)betas.size();
                betas.push_back(std::acos(std::max(-1.0, std::min(1.0, tz / T))));
            }
            const std::pair<int, int> kd{dx * dx + dy * dy + dz * dz, 0};
            if (!dkey.count(kd)) {
                dkey[kd] = (int)dists.size();
                dists.push_back(T);
            }
            opi[2 * o] = bkey[kb];
            opi[2 * o + 1] = dkey[kd];
            const double phi = (dx == 0 && dy == 0) ? 0.0 : std::atan2(ty, tx);
            for (int m = 0; m < p; ++m) ph[(size_t)o * p + m] = std::polar(1.0, m * phi);
        }
        V.hwsz = wsize(p);
        V.hcsz = csize(p, p);
        std::vector<double> Wt((size_t)std::max<size_t>(1, betas.size()) * V.hwsz, 0.0);
        parallel_for((int)betas.size(), [&](int i) { rotation_table(p, betas[i], Wt.data() + (size_t)i * V.hwsz); });
        std::vector<cd> Ct((size_t)std::max<size_t>(1, dists.size()) * V.hcsz);
        parallel_for((int)dists.size(), [&](int i) {
            coax_table(CX_SR, k, dists[i], p, p, alpha[l], alpha[l], Ct.data() + (size_t)i * V.hcsz);
        });
        // --- octant directions: 0..7 M2M into this level (t = X_parent - X_child of child octant o),
        //     8..15 L2L into this level (t = X_child - X_parent of own octant o)
        const int pu = l < L ? P.lv[l + 1].p : 0, pdn = l > lmin ? P.lv[l - 1].p : 0;
        V.hpwo = std::max(p, std::max(pu, pdn));
        V.hwszo = wsize(V.hpwo);
        std::vector<double> Wo((size_t)2 * V.hwszo);
        parallel_for(2, [&](int i) { rotation_table(V.hpwo, std::acos(i == 0 ? c1 : -c1), Wo.data() + (size_t)i * V.hwszo); });
        std::vector<cd> pho((size_t)16 * V.hpwo);
        std::vector<int32_t> boct(16);
        for (int q = 0; q < 16; ++q) {
            const int o = q & 7;
            const double sg = q < 8 ? -1.0 : 1.0;
            const double v[3] = {sg * (((o >> 0) & 1) - 0.5), sg * (((o >> 1) & 1) - 0.5), sg * (((o >> 2) & 1) - 0.5)};
            boct[q] = v[2] > 0 ? 0 : 1;
            const double phi = std::atan2(v[1], v[0]);
            for (int m = 0; m < V.hpwo; ++m) pho[(size_t)q * V.hpwo + m] = std::polar(1.0, m * phi);
        }
        std::vector<cd> Css, Crr;
        if (l < L) {
            // S|S from children at level l+1: |t| = sqrt(3)/2 * side_{l+1}
            Css.resize(csize(p, pu));
            coax_table(CX_SS, k, 0.5 * std::sqrt(3.0) * side * 0.5, p, pu, alpha[l], alpha[l + 1], Css.data());
        }
        if (l > lmin) {
            // R|R from the parent at level l-1: |t| = sqrt(3)/2 * side_l
            Crr.resize(csize(p, pdn));
            coax_table(CX_RR, k, 0.5 * std::sqrt(3.0) * side, p, pdn, alpha[l], alpha[l - 1], Crr.data());
        }
        upload_as<int32_t>(V.hopi, std::vector<double>(opi.begin(), opi.end()), s);
        upload_as<int32_t>(V.hboct, std::vector<double>(boct.begin(), boct.end()), s);
        {
            std::vector<double> oi(32, 0.0);
            for (int q = 0; q < 16; ++q) oi[2 * q] = boct[q];
            upload_as<int32_t>(V.hoinfo, oi, s);
            const std::vector<int32_t> nc = degree_chunks(p, V.hnck_max), mc = m_chunks(p, p, V.hmck_max),
                                       mss = m_chunks(p, pu, V.hmck_ss_max), mrr = m_chunks(p, pdn, V.hmck_rr_max);
            V.hnnck = (int)nc.size() - 1;
            V.hnmck = (int)mc.size() - 1;
            V.hnmck_ss = (int)mss.size() - 1;
            V.hnmck_rr = (int)mrr.size() - 1;
            upload_as<int32_t>(V.hnck, std::vector<double>(nc.begin(), nc.end()), s);
            upload_as<int32_t>(V.hmck, std::vector<double>(mc.begin(), mc.end()), s);
            upload_as<int32_t>(V.hmck_ss, std::vector<double>(mss.begin(), mss.end()), s);
            upload_as<int32_t>(V.hmck_rr, std::vector<double>(mrr.begin(), mrr.end()), s);
        }
        if (f64) {
            upload_as<double>(V.hW, Wt, s);
            upload_as<double>(V.hWo, Wo, s);
            upload_cx<double>(V.hph, ph, s);
            upload_cx<double>(V.hpho, pho, s);
            upload_cx<double>(V.hC, Ct, s);
            upload_cx<double>(V.hCss, Css, s);
            upload_cx<double>(V.hCrr, Crr, s);
        } else {
            upload_as<float>(V.hW, Wt, s);
            upload_as<float>(V.hWo, Wo, s);
            upload_cx<float>(V.hph, ph, s);
            upload_cx<float>(V.hpho, pho, s);
            upload_cx<float>(V.hC, Ct, s);
            upload_cx<float>(V.hCss, Css, s);
            upload_cx<float>(V.hCrr, Crr, s);
        }
    }
    // global scratch for the translation stages whose vectors do not fit in LDS
    const size_t cs = f64 ? sizeof(cx<double>) : sizeof(cx<float>);
    size_t need = 0;
    for (int l = lmin; l <= L; ++l) {
        const Level &V = P.lv[l];
        const int64_t P2 = (int64_t)V.p * V.p;
        const int64_t cols = 3 * (int64_t)P.nrhs_max;
        auto acc_need = [&](int64_t nb, int64_t P2m, int64_t D2) {
            const int mode = f64 ? hf_mode<double>(P2m, D2) : hf_mode<float>(P2m, D2);
            if (mode == 0) need = std::max(need, (size_t)(nb * cols * (2 * P2m + D2)) * cs);
        };
        acc_need(V.nbox, P2, P2);
        if (l < L) {
            const int64_t S2 = (int64_t)P.lv[l + 1].p * P.lv[l + 1].p;
            acc_need(V.nbox, std::max(S2, P2), P2);
        }
        if (l > lmin) {
            const int64_t S2 = (int64_t)P.lv[l - 1].p * P.lv[l - 1].p;
            acc_need(V.nbox, std::max(S2, P2), P2);
        }
    }
    if (need) P.hscratch.alloc(need);
    // per-pair vectors of the pipelined translation sets: room for as many right-hand sides as fit
    // HF_PIPE_BYTES (at least one); wider batches run the pipeline over slices of them
    size_t xneed = 0;
    for (int l = lmin; l <= L; ++l) {
        const Level &V = P.lv[l];
        auto use = [&](int64_t npairs, int ps, int pd) {
            if (std::max(ps, pd) <= HF_PIPE_P) return;
            const size_t per = (size_t)(npairs * 3 * (int64_t)std::max(ps * ps, pd * pd)) * cs;
            const int64_t rc = std::max<int64_t>(1, std::min<int64_t>(P.nrhs_max, (int64_t)(HF_PIPE_BYTES / per)));
            xneed = std::max(xneed, per * (size_t)rc);
        };
        use(V.nff, V.p, V.p);
        if (l < L) use(P.lv[l + 1].nbox, P.lv[l + 1].p, V.p);
        if (l > lmin) use(V.nbox, P.lv[l - 1].p, V.p);
    }
    if (xneed) {
        P.hX1.alloc(xneed);
        P.hX2.alloc(xneed);
    }
}

// ------------------------------------------------------------ launches

// three-launch translation set: npairs pairs (source box src_idx[e] or e, direction dir[e] + dir_add)
// into ndst destinations (pairs of b: dst_ofs[b] .. dst_ofs[b+1], or e = b); mck / nmck / mck_max: the
// |m| chunks of this coaxial shift
template <typename T>
void hf_pipe(Plan &P, int nrhs, hipStream_t s, int64_t npairs, const int32_t *src_idx, const int32_t *dir,
             int dir_add, const int32_t *dinfo, const T *W, int64_t wsz, const cx<T> *ph, int phs, const cx<T> *C,
             int64_t csz, const Level &Vs, const Level &Vd, const DevBuf &mck, int nmck, int mck_max, int64_t ndst,
             const int32_t *dst_ofs, int accumulate, const cx<T> *S, cx<T> *D) {
    if (npairs == 0 || ndst == 0) return;
    const int ps = Vs.p, pd = Vd.p;
    if (Vs.hnck_max > HF_CHUNK_MAX || Vd.hnck_max > HF_CHUNK_MAX || mck_max > HF_CHUNK_MAX)
        throw Status{FMB_EINVAL, "translation chunk larger than the kernels hold"};
    cx<T> *X1 = P.hX1.as<cx<T>>(), *X2 = P.hX2.as<cx<T>>();
    // right-hand sides per slice: what the scratch holds for this set
    const size_t per = (size_t)npairs * 3 * (size_t)std::max(ps * ps, pd * pd) * sizeof(cx<T>);
    const int rc = (int)std::max<size_t>(1, std::min<size_t>((size_t)nrhs, std::min(P.hX1.bytes, P.hX2.bytes) / per));
    if ((size_t)rc * per > std::min(P.hX1.bytes, P.hX2.bytes))
        throw Status{FMB_EINVAL, "pipeline scratch smaller than one right-hand side"};
    const int64_t S2 = (int64_t)ps * ps, D2 = (int64_t)pd * pd;
    for (int r0 = 0; r0 < nrhs; r0 += rc) {
        const int nr = std::min(rc, nrhs - r0);
        // right-hand side r0 of every box starts r0 * 3 p^2 into the box's block
        const cx<T> *Sr = S + (int64_t)r0 * 3 * S2;
        cx<T> *Dr = D + (int64_t)r0 * 3 * D2;
        k_hf_fwd<T><<<dim3((unsigned)npairs, (unsigned)nr, (unsigned)Vs.hnnck), HTPB,
                      3 * (size_t)Vs.hnck_max * sizeof(cx<T>), s>>>(src_idx, dir, dir_add, dinfo, W, wsz, ph, phs,
                                                                    Vs.hnck.as<int32_t>(), ps, P.nrhs_max, nr, Sr, X1);
        FMB_LAUNCH_CHECK();
        k_hf_coax<T><<<dim3((unsigned)npairs, (unsigned)nr, (unsigned)nmck), HTPB,
                       3 * (size_t)mck_max * sizeof(cx<T>), s>>>(dir, dir_add, dinfo, C, csz, mck.as<int32_t>(), ps,
                                                                  pd, nr, X1, X2);
        FMB_LAUNCH_CHECK();
        k_hf_back<T><<<dim3((unsigned)ndst, (unsigned)nr, (unsigned)Vd.hnnck), HTPB,
                       3 * (size_t)Vd.hnck_max * sizeof(cx<T>), s>>>(dst_ofs, dir, dir_add, dinfo, W, wsz, ph, phs,
                                                                     Vd.hnck.as<int32_t>(), pd, P.nrhs_max, nr,
                                                                     accumulate, X2, Dr);
        FMB_LAUNCH_CHECK();
    }
}

template <typename T>
void hf_m2m(Plan &P, int l, int nrhs, hipStream_t s) {
    Level &V = P.lv[l], &Cv = P.lv[l + 1];
    const int ps = Cv.p, pd = V.p;
    if (std::max(ps, pd) > HF_PIPE_P) {
        hf_pipe<T>(P, nrhs, s, Cv.nbox, nullptr, Cv.octant.as<int32_t>(), 0, V.hoinfo.as<int32_t>(), V.hWo.as<T>(),
                   V.hwszo, V.hpho.as<cx<T>>(), V.hpwo, V.hCss.as<cx<T>>(), 0, Cv, V, V.hmck_ss, V.hnmck_ss,
                   V.hmck_ss_max, V.nbox, V.child_start.as<int32_t>(), 0, Cv.M.as<cx<T>>(), V.M.as<cx<T>>());
        return;
    }
    const int64_t S2 = (int64_t)ps * ps, D2 = (int64_t)pd * pd, P2m = std::max(S2, D2);
    const int mode = hf_mode<T>(P2m, D2);
    const int ch = mode == 3 ? 3 : 1;
    const dim3 grid((unsigned)V.nbox, (unsigned)(3 * nrhs / ch));
    const size_t sh = mode ? hf_lds<T>(ch, P2m, D2) : 0;
    auto args = std::make_tuple(V.child_start.as<int32_t>(), Cv.octant.as<int32_t>(), V.hWo.as<T>(), V.hwszo,
                                V.hboct.as<int32_t>(), V.hpho.as<cx<T>>(), V.hpwo, V.hCss.as<cx<T>>(), ps, pd,
                                P.nrhs_max, Cv.M.as<cx<T>>(), V.M.as<cx<T>>(), P.hscratch.as<cx<T>>());
    auto go = [&](auto kern) { std::apply([&](auto... a) { kern<<<grid, HTPB, sh, s>>>(a...); }, args); };
    if (mode == 3) go(k_hf_m2m<T, 3, false>);
    else if (mode == 1) go(k_hf_m2m<T, 1, false>);
    else go(k_hf_m2m<T, 1, true>);
    FMB_LAUNCH_CHECK();
}

template <typename T>
void hf_m2l(Plan &P, int l, int nrhs, hipStream_t s) {
    Level &V = P.lv[l];
    if (V.nff == 0) {
        // no far-field pairs: the level's local expansions start at zero
        const int64_t m = V.nbox * P.nrhs_max * 3 * (int64_t)V.p * V.p;
        k_hf_zero<T><<<(unsigned)((m + HTPB - 1) / HTPB), HTPB, 0, s>>>(V.L.as<cx<T>>(), m);
        FMB_LAUNCH_CHECK();
        return;
    }
    const int p = V.p;
    if (p > HF_PIPE_P) {
        hf_pipe<T>(P, nrhs, s, V.nff, V.ff_src.as<int32_t>(), V.ff_op.as<int32_t>(), 0, V.hopi.as<int32_t>(),
                   V.hW.as<T>(), V.hwsz, V.hph.as<cx<T>>(), p, V.hC.as<cx<T>>(), V.hcsz, V, V, V.hmck, V.hnmck,
                   V.hmck_max, V.nbox, V.ff_ofs.as<int32_t>(), 0, V.M.as<cx<T>>(), V.L.as<cx<T>>());
        return;
    }
    if (p <= HFW_PMAX && hfw_lds<T>(p) <= HFW_LDS_MAX) {
        const int J = (p * p + 63) / 64;
        const size_t sh = hfw_lds<T>(p);
        auto go = [&](auto kern) {
            if (sh > 64 * 1024)
                FMB_CHECK_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)HFW_LDS_MAX));
            kern<<<dim3((unsigned)V.nbox, (unsigned)nrhs), 256, sh, s>>>(
                V.ff_ofs.as<int32_t>(), V.ff_src.as<int32_t>(), V.ff_op.as<int32_t>(), V.hopi.as<int32_t>(), V.hW.as<T>(),
                V.hwsz, V.hph.as<cx<T>>(), V.hC.as<cx<T>>(), V.hcsz, p, P.nrhs_max, V.M.as<cx<T>>(), V.L.as<cx<T>>());
        };
        if (J <= 2) go(k_hf_m2l_w<T, 2>);
        else if (J <= 3) go(k_hf_m2l_w<T, 3>);
        else if (J <= 5) go(k_hf_m2l_w<T, 5>);
        else go(k_hf_m2l_w<T, 7>);
        FMB_LAUNCH_CHECK();
        return;
    }
    const int64_t P2 = (int64_t)p * p;
    const int mode = hf_mode<T>(P2, P2);
    const int ch = mode == 3 ? 3 : 1;
    const dim3 grid((unsigned)V.nbox, (unsigned)(3 * nrhs / ch));
    const size_t sh = mode ? hf_lds<T>(ch, P2, P2) : 0;
    auto args = std::make_tuple(V.ff_ofs.as<int32_t>(), V.ff_src.as<int32_t>(), V.ff_op.as<int32_t>(),
                                V.hopi.as<int32_t>(), V.hW.as<T>(), V.hwsz, V.hph.as<cx<T>>(), V.hC.as<cx<T>>(),
                                V.hcsz, p, P.nrhs_max, V.M.as<cx<T>>(), V.L.as<cx<T>>(), P.hscratch.as<cx<T>>());
    auto go = [&](auto kern) { std::apply([&](auto... a) { kern<<<grid, HTPB, sh, s>>>(a...); }, args); };
    if (mode == 3) go(k_hf_m2l<T, 3, false>);
    else if (mode == 1) go(k_hf_m2l<T, 1, false>);
    else go(k_hf_m2l<T, 1, true>);
    FMB_LAUNCH_CHECK();
}

template <typename T>
void hf_l2l(Plan &P, int l, int nrhs, hipStream_t s) {
    Level &V = P.lv[l], &U = P.lv[l - 1];
    const int ps = U.p, pd = V.p;
    if (std::max(ps, pd) > HF_PIPE_P) {
        hf_pipe<T>(P, nrhs, s, V.nbox, V.parent.as<int32_t>(), V.octant.as<int32_t>(), 8, V.hoinfo.as<int32_t>(),
                   V.hWo.as<T>(), V.hwszo, V.hpho.as<cx<T>>(), V.hpwo, V.hCrr.as<cx<T>>(), 0, U, V, V.hmck_rr,
                   V.hnmck_rr, V.hmck_rr_max, V.nbox, nullptr, 1, U.L.as<cx<T>>(), V.L.as<cx<T>>());
        return;
    }
    const int64_t S2 = (int64_t)ps * ps, D2 = (int64_t)pd * pd, P2m = std::max(S2, D2);
    const int mode = hf_mode<T>(P2m, D2);
    const int ch = mode == 3 ? 3 : 1;
    const dim3 grid((unsigned)V.nbox, (unsigned)(3 * nrhs / ch));
    const size_t sh = mode ? hf_lds<T>(ch, P2m, D2) : 0;
    auto args = std::make_tuple(V.parent.as<int32_t>(), V.octant.as<int32_t>(), V.hWo.as<T>(), V.hwszo,
                                V.hboct.as<int32_t>(), V.hpho.as<cx<T>>(), V.hpwo, V.hCrr.as<cx<T>>(), ps, pd,
                                P.nrhs_max, U.L.as<cx<T>>(), V.L.as<cx<T>>(), P.hscratch.as<cx<T>>());
    auto go = [&](auto kern) { std::apply([&](auto... a) { kern<<<grid, HTPB, sh, s>>>(a...); }, args); };
    if (mode == 3) go(k_hf_l2l<T, 3, false>);
    else if (mode == 1) go(k_hf_l2l<T, 1, false>);
    else go(k_hf_l2l<T, 1, true>);
    FMB_LAUNCH_CHECK();
}

template void hf_m2m<float>(Plan &, int, int, hipStream_t);
template void hf_m2m<double>(Plan &, int, int, hipStream_t);
template void hf_m2l<float>(Plan &, int, int, hipStream_t);
template void hf_m2l<double>(Plan &, int, int, hipStream_t);
template void hf_l2l<float>(Plan &, int, int, hipStream_t);
template void hf_l2l<double>(Plan &, int, int, hipStream_t);

}  // namespace fmb
