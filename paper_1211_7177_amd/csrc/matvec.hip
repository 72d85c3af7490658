// One fast-multipole matvec y = Op_k(a, b) (Sec. 2.2, Steps 1-4).
//
// Each output channel c = x, y, z is a Helmholtz potential of sources that
// carry a monopole and a dipole:
//   y_c(s_alpha) = sum_beta [ sigma_{beta,c} g(s_beta, s_alpha) + q_{beta,c} . grad' g(s_beta, s_alpha) ],
//   sigma_{beta,c} = w b_c,   q_{beta,c} = w (n_c a - a_c n - (n . a) e_c),
// which is the kernel n (grad'g . a) - (n . grad'g) a - grad'g (n . a) + g b of
// eq. 2.12 written per component.  Hence
//   Step 1 (eqs. 2.18-2.19): M_nm,c = i k sum_beta [sigma_c R_n^-m + q_c . grad R_n^-m](s_beta - X),
//   Step 2 (eq. 2.20): S|S to the parent, Step 3 (eq. 2.21): S|R over FF plus
//   R|R from the parent, Step 4 (eq. 2.23): y_c = sum L_nm,c R_n^m(s - X) plus
//   the near sum over the leaf and its neighbours.
// Gradients of R_n^m use the recurrences that follow from the plane-wave form
// of R (cos(theta) and sin(theta) e^{+-i phi} times Y_n^m shift n by one):
//   d_z R_n^m        = k [ -A_n^m R_{n+1}^m     + B_n^m R_{n-1}^m ]
//   (d_x + i d_y) R  = k [ -C_n^m R_{n+1}^{m+1} + D_n^m R_{n-1}^{m+1} ]
//   (d_x - i d_y) R  = k [ -E_n^m R_{n+1}^{m-1} + F_n^m R_{n-1}^{m-1} ]
#include <array>
#include <map>

#include "basis.h"
#include "plan.h"

namespace fmb {

namespace {

constexpr int TPB = 256;

template <typename T>
__device__ inline cx<T> tc(cx<double> z) { return mk((T)z.re, (T)z.im); }

// ---------------------------------------------------------------- gather
template <typename T>
__global__ void k_gather_src(const cx<T> *__restrict__ a, const cx<T> *__restrict__ b, const int32_t *__restrict__ perm,
                             const double *__restrict__ sw, const double *__restrict__ snrm, int64_t n, int nrhs,
                             cx<T> *__restrict__ src) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    const T w = (T)sw[i];
    const T nx = (T)snrm[3 * i], ny = (T)snrm[3 * i + 1], nz = (T)snrm[3 * i + 2];
    for (int r = 0; r < nrhs; ++r) {
        const cx<T> *A = a + ((int64_t)r * n + u) * 3;
        const cx<T> *B = b + ((int64_t)r * n + u) * 3;
        cx<T> *o = src + ((int64_t)r * n + i) * 7;
        cx<T> wa0 = w * A[0], wa1 = w * A[1], wa2 = w * A[2];
        o[0] = wa0;
        o[1] = wa1;
        o[2] = wa2;
        o[3] = w * B[0];
        o[4] = w * B[1];
        o[5] = w * B[2];
        o[6] = nx * wa0 + ny * wa1 + nz * wa2;
    }
}

template <typename T>
__global__ void k_scatter_out(const cx<T> *__restrict__ ys, const int32_t *__restrict__ perm, int64_t n, int nrhs,
                              cx<T> *__restrict__ y) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    for (int r = 0; r < nrhs; ++r)
        for (int c = 0; c < 3; ++c) y[((int64_t)r * n + u) * 3 + c] = ys[((int64_t)r * n + i) * 3 + c];
}

// MI355X dispatches consecutive workgroups to its 8 XCDs in turn.  Tiles are
// listed operator by operator; renumbering block i to tile (i % 8) * chunk + i / 8
// gives each XCD a contiguous run of tiles, so the tiles that share an operator
// share one L2.  The grid is padded to a multiple of 8; spare blocks exit.
__device__ inline int xcd_tile(int i, int ntiles) {
    const int chunk = (ntiles + 7) / 8;
    return (i % 8) * chunk + i / 8;
}

// ---------------------------------------------------------------- P2M
// One block per leaf.  For a batch of the leaf's nodes the block first builds
// the table R_n^m(s - X), n <= p, in LDS (one thread per (node, m) column;
// entry (p+1)^2 of each node's table is a zero that stands for the terms the
// gradient recurrence lacks), then G = blockDim / p^2 thread groups each take
// every G-th node of the batch and accumulate all three channels of one
// coefficient; the groups are summed in LDS at the end (fixed order, so the
// result is deterministic).  The gradient of R_n^{-m} is
//   d_z = k (c0 R[i0] + c1 R[i1]),  d_+ = k (c2 R[i2] + c3 R[i3]),  d_- = k (c4 R[i4] + c5 R[i5]),
//   grad = ((d_+ + d_-) / 2, (d_+ - d_-) / 2i, d_z),
// with coefficients and indices from the plan's table; k multiplies the whole
// gradient part once per coefficient after the node loop.
constexpr int P2M_SLOTS = 3;     // coefficients per thread when p^2 > blockDim (orders up to 27)
constexpr int P2M_SLOTS_MAX = 7; // leaf orders 28..40 (7 x 256 >= 40^2)

template <typename T, int SLOTS>
__global__ void __launch_bounds__(TPB) k_p2m(const int32_t *__restrict__ start, const double *__restrict__ center,
                                             const double *__restrict__ spts, const double *__restrict__ snrm,
                                             const cx<T> *__restrict__ src, int64_t n, int p, double k_re, double k_im,
                                             const double *__restrict__ inv_alpha, const T *__restrict__ tab,
                                             const int32_t *__restrict__ gix, int nrhs, int nrhs_max, int batch,
                                             cx<T> *__restrict__ M) {
    extern __shared__ unsigned char smem[];
    const int N = p;                                  // degrees 0..p for the gradients
    const int NN = (N + 1) * (N + 1);
    const int NT = NN + 1;                            // per-node table incl. the zero entry
    const int P2 = p * p;
    const BasisTab<T> bt = basis_tab(tab, gix, N, P2);
    const int G = P2 <= (int)blockDim.x ? (int)blockDim.x / P2 : 1;   // node groups
    const int grp = P2 <= (int)blockDim.x ? (int)threadIdx.x / P2 : 0;
    cx<T> *red = reinterpret_cast<cx<T> *>(smem);                       // [G][P2][3] (G > 1)
    cx<T> *Rb = red + (G > 1 ? G * P2 * 3 : 0);                         // [batch][NT]
    cx<T> *jb = Rb + batch * NT;                                        // [batch][N+1]
    cx<T> *sv = jb + batch * (N + 1);                                   // [batch][7] node densities
    T *dd = reinterpret_cast<T *>(sv + batch * 7);                      // [batch][3] cos th, sin th e^{i ph}
    T *nvs = dd + batch * 3;                                            // [batch][3] normals
    const int box = blockIdx.x;
    const int s0 = start[box], s1 = start[box + 1];
    const double X[3] = {center[3 * box], center[3 * box + 1], center[3 * box + 2]};
    const cx<T> k = mk((T)k_re, (T)k_im);
    // a leaf that fits one batch builds its tables once for all right-hand sides
    const bool one = s1 - s0 <= batch;
    for (int r = 0; r < nrhs; ++r) {
        cx<T> accb[SLOTS][3], accg[SLOTS][3];
        for (int u = 0; u < SLOTS; ++u)
            for (int c = 0; c < 3; ++c) accb[u][c] = accg[u][c] = mk(T(0), T(0));
        for (int b0 = s0; b0 < s1; b0 += batch) {
            const int nb = min(batch, s1 - b0);
            __syncthreads();
            if (!one || r == 0) {
                for (int t = threadIdx.x; t < nb; t += blockDim.x) {
                    const int i = b0 + t;
                    double d[3];
                    for (int q = 0; q < 3; ++q) d[q] = spts[3 * (int64_t)i + q] - X[q];
                    const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                    const double ir = rr > 0 ? 1.0 / rr : 0.0;
                    dd[t * 3] = rr > 0 ? (T)(d[2] * ir) : T(1);
                    dd[t * 3 + 1] = (T)(d[0] * ir);
                    dd[t * 3 + 2] = (T)(d[1] * ir);
                    sph_bessel_j(mk((T)(k_re * rr), (T)(k_im * rr)), N, jb + t * (N + 1));
                    Rb[t * NT + NN] = mk(T(0), T(0));
                    for (int q = 0; q < 3; ++q) nvs[t * 3 + q] = (T)snrm[3 * (int64_t)i + q];
                }
                __syncthreads();
                for (int t = threadIdx.x; t < nb * (N + 1); t += blockDim.x) {
                    const int i = t / (N + 1), m = t % (N + 1);
                    regular_column<T>(dd[3 * i], mk(dd[3 * i + 1], dd[3 * i + 2]), jb + i * (N + 1), bt, m,
                                      Rb + i * NT);
                }
            }
            for (int t = threadIdx.x; t < nb * 7; t += blockDim.x)
                sv[t] = src[((int64_t)r * n + b0) * 7 + t];
            __syncthreads();
            for (int u = 0; u < SLOTS; ++u) {
                const int idx = (G > 1) ? ((int)threadIdx.x % P2) : (int)threadIdx.x + u * (int)blockDim.x;
                if (idx >= P2 || grp >= G || (G > 1 && u > 0)) break;
                int ix[7];
                T co[6];
                for (int q = 0; q < 7; ++q) ix[q] = bt.gix[idx * 7 + q];
                for (int q = 0; q < 6; ++q) co[q] = bt.gco[idx * 6 + q];
                for (int i = grp; i < nb; i += G) {
                    const cx<T> *R = Rb + i * NT;
                    const cx<T> Rv = R[ix[6]];                                  // R_n^{-m}
                    const cx<T> dz = co[0] * R[ix[0]] + co[1] * R[ix[1]];
                    const cx<T> dp = co[2] * R[ix[2]] + co[3] * R[ix[3]];
                    const cx<T> dm = co[4] * R[ix[4]] + co[5] * R[ix[5]];
                    const cx<T> df = dp - dm;
                    const cx<T> g[3] = {T(0.5) * (dp + dm), mk(T(0.5) * df.im, T(-0.5) * df.re), dz};   // grad / k
                    const cx<T> *sr = sv + i * 7;
                    const T nv[3] = {nvs[3 * i], nvs[3 * i + 1], nvs[3 * i + 2]};
                    const cx<T> aG = sr[0] * g[0] + sr[1] * g[1] + sr[2] * g[2];
                    const cx<T> nG = nv[0] * g[0] + nv[1] * g[1] + nv[2] * g[2];
                    for (int c = 0; c < 3; ++c) {
                        accb[u][c] += sr[3 + c] * Rv;
                        accg[u][c] += nv[c] * aG - sr[c] * nG - sr[6] * g[c];
                    }
                }
            }
        }
        cx<T> acc[SLOTS][3];
        for (int u = 0; u < SLOTS; ++u)
            for (int c = 0; c < 3; ++c) acc[u][c] = accb[u][c] + k * accg[u][c];
        cx<T> *Mo = M + ((int64_t)box * nrhs_max + r) * 3 * P2;
        if (G > 1) {
            // sum the node groups in LDS
            __syncthreads();
            if (grp < G)
                for (int c = 0; c < 3; ++c) red[(grp * P2 + (threadIdx.x % P2)) * 3 + c] = acc[0][c];
            __syncthreads();
            if ((int)threadIdx.x < P2) {
                const int idx = threadIdx.x;
                int nn = 0;
                while ((nn + 1) * (nn + 1) <= idx) ++nn;
                const cx<T> sc = mk((T)(-k_im * inv_alpha[nn]), (T)(k_re * inv_alpha[nn]));   // i k / alpha_n
                for (int c = 0; c < 3; ++c) {
                    cx<T> s = mk(T(0), T(0));
                    for (int g2 = 0; g2 < G; ++g2) s += red[(g2 * P2 + idx) * 3 + c];
                    Mo[c * P2 + idx] = sc * s;
                }
            }
        } else {
            for (int u = 0; u < SLOTS; ++u) {
                const int idx = threadIdx.x + u * blockDim.x;
                if (idx >= P2) break;
                int nn = 0;
                while ((nn + 1) * (nn + 1) <= idx) ++nn;
                const cx<T> sc = mk((T)(-k_im * inv_alpha[nn]), (T)(k_re * inv_alpha[nn]));   // i k / alpha_n
                for (int c = 0; c < 3; ++c) Mo[c * P2 + idx] = sc * acc[u][c];
            }
        }
    }
}

// ---------------------------------------------------------------- L2P
// RC right-hand sides per block (blockIdx.y = chunk of RC): each node's basis
// values are evaluated once and contracted with the RC local expansions.
template <typename T, int RC>
__global__ void __launch_bounds__(64) k_l2p(const int32_t *__restrict__ start, const double *__restrict__ center,
                                            const double *__restrict__ spts, int64_t n, int p, double k_re, double k_im,
                                            const double *__restrict__ inv_alpha, const T *__restrict__ tab,
                                            int nrhs, int nrhs_max, const cx<T> *__restrict__ Lc,
                                            cx<T> *__restrict__ ys) {
    extern __shared__ unsigned char smem[];
    const int P2 = p * p;
    const BasisTab<T> bt = basis_tab(tab, (const int32_t *)nullptr, p, P2);
    cx<T> *Ls = reinterpret_cast<cx<T> *>(smem);        // [RC][3][P2]
    cx<T> *jb = Ls + RC * 3 * P2;                        // [64][p]
    const int box = blockIdx.x, r0 = blockIdx.y * RC;
    const int rcn = min(RC, nrhs - r0);
    const int s0 = start[box], s1 = start[box + 1];
    for (int t = threadIdx.x; t < RC * 3 * P2; t += blockDim.x) {
        const int rr = t / (3 * P2), e = t % (3 * P2);
        const int idx = e % P2;
        int nn = 0;
        while ((nn + 1) * (nn + 1) <= idx) ++nn;
        Ls[t] = rr < rcn ? (T)inv_alpha[nn] * Lc[((int64_t)box * nrhs_max + r0 + rr) * 3 * P2 + e] : mk(T(0), T(0));
    }
    __syncthreads();
    const double X[3] = {center[3 * box], center[3 * box + 1], center[3 * box + 2]};
    for (int i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
        double d[3];
        for (int q = 0; q < 3; ++q) d[q] = spts[3 * (int64_t)i + q] - X[q];
        const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double ir = rr > 0 ? 1.0 / rr : 0.0;
        cx<T> *J = jb + threadIdx.x * p;
        sph_bessel_j(mk((T)(k_re * rr), (T)(k_im * rr)), p - 1, J);
        const T x = rr > 0 ? (T)(d[2] * ir) : T(1);
        const cx<T> w = mk((T)(d[0] * ir), (T)(d[1] * ir));
        cx<T> acc[RC][3];
#pragma unroll
        for (int q = 0; q < RC; ++q)
            for (int c = 0; c < 3; ++c) acc[q][c] = mk(T(0), T(0));
        cx<T> wm = mk(T(1), T(0));
        for (int m = 0; m < p; ++m) {
            if (m > 0) wm = wm * w;
            const T qmm = bt.qmm[m];
            const T sgn = (m & 1) ? T(-1) : T(1);
            T q2 = 0, q1 = qmm;
            for (int nn = m; nn < p; ++nn) {
                T q;
                if (nn == m) q = qmm;
                else if (nn == m + 1) q = bt.q1[m] * x * qmm;
                else q = bt.la[nn * (bt.N + 1) + m] * (x * q1 - bt.lb[nn * (bt.N + 1) + m] * q2);
                if (nn > m) {
                    q2 = q1;
                    q1 = q;
                }
                const cx<T> Y = (sgn * q) * wm;
                const cx<T> Rp = J[nn] * Y;
                const cx<T> Rm = J[nn] * conj(Y);
#pragma unroll
                for (int rq = 0; rq < RC; ++rq) {
                    const cx<T> *L = Ls + rq * 3 * P2;
                    for (int c = 0; c < 3; ++c) acc[rq][c] += L[c * P2 + nn * nn + nn + m] * Rp;
                    if (m > 0)
                        for (int c = 0; c < 3; ++c) acc[rq][c] += L[c * P2 + nn * nn + nn - m] * Rm;
                }
            }
        }
#pragma unroll
        for (int rq = 0; rq < RC; ++rq)
            if (rq < rcn)
                for (int c = 0; c < 3; ++c) ys[((int64_t)(r0 + rq) * n + i) * 3 + c] = acc[rq][c];
    }
}

// ---------------------------------------------------------------- P2P
// One block per leaf.  Targets on lanes; when a leaf holds fewer targets
// than the block has threads, the sources are split into S slices handled by
// the spare threads and the slices are summed in LDS at the end.
constexpr int P2P_TILE = 256;

template <typename T>
struct SrcTile {
    double pos[P2P_TILE][3];
    T nrm[P2P_TILE][3];
    int32_t tri[P2P_TILE];
    cx<T> rec[P2P_TILE][7];
};

template <typename T>
__global__ void __launch_bounds__(TPB) k_p2p(const int32_t *__restrict__ start, const int32_t *__restrict__ nbr,
                                             const double *__restrict__ spts, const double *__restrict__ snrm,
                                             const int32_t *__restrict__ stri, const cx<T> *__restrict__ src, int64_t n,
                                             double k_re, double k_im, double rcut2, cx<T> *__restrict__ ys) {
    __shared__ SrcTile<T> tile;
    __shared__ int32_t nb_start[28], nb_box[27];
    __shared__ int n_nb;
    __shared__ cx<T> red[TPB][3];
    const int box = blockIdx.x, r = blockIdx.y;
    const int t0 = start[box], t1 = start[box + 1];
    const int nt = t1 - t0;
    if (threadIdx.x == 0) {
        int c = 0, tot = 0;
        for (int s = 0; s < 27; ++s) {
            int q = nbr[box * 27 + s];
            if (q >= 0) {
                nb_box[c] = q;
                nb_start[c] = tot;
                tot += start[q + 1] - start[q];
                ++c;
            }
        }
        nb_start[c] = tot;
        n_nb = c;
    }
    __syncthreads();
    const int ns_total = nb_start[n_nb];
    const T kr = (T)k_re, ki = (T)k_im;
    const T inv4pi = T(0.07957747154594766788);
    for (int tc0 = 0; tc0 < nt; tc0 += TPB) {
        const int ntc = min(TPB, nt - tc0);
        const int S = TPB / ntc;                 // source slices
        const int ti = threadIdx.x % ntc, sl = threadIdx.x / ntc;
        const bool active = sl < S;
        const int64_t ig = t0 + tc0 + ti;
        double tp[3] = {0, 0, 0};
        int32_t ttri = -1;
        if (active) {
            for (int q = 0; q < 3; ++q) tp[q] = spts[3 * ig + q];
            ttri = stri[ig];
        }
        cx<T> acc[3] = {mk(T(0), T(0)), mk(T(0), T(0)), mk(T(0), T(0))};
        for (int base = 0; base < ns_total; base += P2P_TILE) {
            const int cnt = min(P2P_TILE, ns_total - base);
            __syncthreads();
            for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
                const int u = base + j;
                int b = 0;
                while (nb_start[b + 1] <= u) ++b;
                const int64_t sidx = start[nb_box[b]] + (u - nb_start[b]);
                for (int q = 0; q < 3; ++q) {
                    tile.pos[j][q] = spts[3 * sidx + q];
                    tile.nrm[j][q] = (T)snrm[3 * sidx + q];
                }
                tile.tri[j] = stri[sidx];
                const cx<T> *sr = src + ((int64_t)r * n + sidx) * 7;
                for (int q = 0; q < 7; ++q) tile.rec[j][q] = sr[q];
            }
            __syncthreads();
            if (!active) continue;
            for (int j = sl; j < cnt; j += S) {
                if (tile.tri[j] == ttri) continue;
                const T dx = (T)(tile.pos[j][0] - tp[0]), dy = (T)(tile.pos[j][1] - tp[1]),
                        dz = (T)(tile.pos[j][2] - tp[2]);
                const T R2 = dx * dx + dy * dy + dz * dz;
                if (R2 > rcut2) continue;       // damped below the cutoff (local-only lossy plans)
                const T iR = fast_rsqrt(R2);
                const T R = R2 * iR;
                T sn, cs;
                fast_sincos(kr * R, &sn, &cs);
                const T ex = ki != T(0) ? fast_exp(-ki * R) : T(1);
                const cx<T> e = mk(ex * cs, ex * sn);
                const cx<T> g = (inv4pi * iR) * e;
                // f = (i k R - 1) e / (4 pi R^3)
                const cx<T> ikR1 = mk(-ki * R - T(1), kr * R);
                const cx<T> f = (inv4pi * iR * iR * iR) * (ikR1 * e);
                const T nx = tile.nrm[j][0], ny = tile.nrm[j][1], nz = tile.nrm[j][2];
                const T v = nx * dx + ny * dy + nz * dz;
                const cx<T> *rc = tile.rec[j];
                const cx<T> u = dx * rc[0] + dy * rc[1] + dz * rc[2];
                const cx<T> tx = nx * u - v * rc[0] - dx * rc[6];
                const cx<T> ty = ny * u - v * rc[1] - dy * rc[6];
                const cx<T> tz = nz * u - v * rc[2] - dz * rc[6];
                acc[0] += f * tx + g * rc[3];
                acc[1] += f * ty + g * rc[4];
                acc[2] += f * tz + g * rc[5];
            }
        }
        __syncthreads();
        for (int c = 0; c < 3; ++c) red[threadIdx.x][c] = acc[c];
        __syncthreads();
        if (threadIdx.x < ntc) {
            cx<T> s[3] = {mk(T(0), T(0)), mk(T(0), T(0)), mk(T(0), T(0))};
            for (int q = 0; q < S; ++q)
                for (int c = 0; c < 3; ++c) s[c] += red[q * ntc + threadIdx.x][c];
            cx<T> *o = ys + ((int64_t)r * n + t0 + tc0 + threadIdx.x) * 3;
            for (int c = 0; c < 3; ++c) o[c] += s[c];
        }
    }
}

// FP32 near field, one block per leaf in Morton order.  Consecutive blocks go
// to different XCDs; giving each XCD contiguous runs of leaves cuts the L2-miss
// traffic (52 -> 12 MB per launch on the 60k-node torus) but unbalances the
// load and is slower, and the kernel is bound by its arithmetic.  Source
// records are packed into six 16-byte LDS words per source: position relative
// to the target leaf's centre (FP32; the leaf and its neighbours span a few
// leaf widths, so the difference keeps FP32 relative accuracy) with the
// triangle id, the normal, and the seven density values.  The transcendentals
// go straight to the hardware units with the scale folded into the constants:
// v_sin/v_cos take revolutions (kR / 2 pi), v_exp takes a base-2 exponent
// (-Im k R log2 e); the LOSSY = false instance (real k) skips the decay
// factor.  Same-triangle pairs are masked, not branched around, so the source
// loop unrolls.
struct __attribute__((aligned(16))) SrcHdr32 {
    float x, y, z;
    int32_t tri;
    float nx, ny, nz, pad;
};

// RC right-hand sides per block (blockIdx.y = chunk of RC): the pair geometry,
// the transcendentals and g, f are computed once per pair and applied to all
// RC density sets.  The source tile shrinks as RC grows to keep LDS near 32 KB.
template <int RC>
struct P2PTile {
    static constexpr int TS = RC == 1 ? 256 : (RC == 2 ? 128 : 64);
};

template <bool LOSSY, int RC, bool CUT = false>
__global__ void __launch_bounds__(TPB) k_p2p32(int nleaf, int nrhs, const int32_t *__restrict__ start,
                                               const int32_t *__restrict__ nbr,
                                               const double *__restrict__ center, const double *__restrict__ spts,
                                               const double *__restrict__ snrm, const int32_t *__restrict__ stri,
                                               const cx<float> *__restrict__ src, int64_t n, double k_re,
                                               double k_im, float rcut2, cx<float> *__restrict__ ys) {
    constexpr int TS = P2PTile<RC>::TS;
    __shared__ SrcHdr32 hdr[TS];
    __shared__ __attribute__((aligned(16))) cx<float> rec[TS][RC][8];   // a[3], b[3], n.a, unused
    __shared__ int32_t sid[TS];
    __shared__ int32_t nb_start[28], nb_box[27];
    __shared__ int n_nb;
    __shared__ cx<float> red[TPB][3];
    const int box = blockIdx.x, r0 = blockIdx.y * RC;
    if (box >= nleaf) return;
    const int rcn = min(RC, nrhs - r0);
    const int t0 = start[box], t1 = start[box + 1];
    const int nt = t1 - t0;
    const double c0x = center[3 * box], c0y = center[3 * box + 1], c0z = center[3 * box + 2];
    if (threadIdx.x == 0) {
        int c = 0, tot = 0;
        for (int s = 0; s < 27; ++s) {
            int q = nbr[box * 27 + s];
            if (q >= 0) {
                nb_box[c] = q;
                nb_start[c] = tot;
                tot += start[q + 1] - start[q];
                ++c;
            }
        }
        nb_start[c] = tot;
        n_nb = c;
    }
    __syncthreads();
    const int ns_total = nb_start[n_nb];
    const float krev = (float)(k_re * 0.15915494309189533577);        // k_re / (2 pi)
    const float kexp = (float)(-k_im * 1.44269504088896340736);       // -k_im log2(e)
    const float kr = (float)k_re, ki = (float)k_im;
    const float inv4pi = 0.07957747154594766788f;
    for (int tc0 = 0; tc0 < nt; tc0 += TPB) {
        const int ntc = min(TPB, nt - tc0);
        const int S = TPB / ntc;
        const int ti = threadIdx.x % ntc, sl = threadIdx.x / ntc;
        const bool active = sl < S;
        const int64_t ig = t0 + tc0 + ti;
        float tx = 0.f, ty = 0.f, tz = 0.f;
        int32_t ttri = -1;
        if (active) {
            tx = (float)(spts[3 * ig] - c0x);
            ty = (float)(spts[3 * ig + 1] - c0y);
            tz = (float)(spts[3 * ig + 2] - c0z);
            ttri = stri[ig];
        }
        cx<float> acc[RC][3];
#pragma unroll
        for (int rr = 0; rr < RC; ++rr)
            for (int c = 0; c < 3; ++c) acc[rr][c] = mk(0.f, 0.f);
        for (int base = 0; base < ns_total; base += TS) {
            const int cnt = min(TS, ns_total - base);
            __syncthreads();
            for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
                const int u = base + j;
                int b = 0;
                while (nb_start[b + 1] <= u) ++b;
                const int64_t sidx = start[nb_box[b]] + (u - nb_start[b]);
                SrcHdr32 q;
                q.x = (float)(spts[3 * sidx] - c0x);
                q.y = (float)(spts[3 * sidx + 1] - c0y);
                q.z = (float)(spts[3 * sidx + 2] - c0z);
                q.tri = stri[sidx];
                q.nx = (float)snrm[3 * sidx];
                q.ny = (float)snrm[3 * sidx + 1];
                q.nz = (float)snrm[3 * sidx + 2];
                q.pad = 0.f;
                hdr[j] = q;
                sid[j] = (int32_t)sidx;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < cnt * RC * 8; e += blockDim.x) {
                const int w = e % 8, rr = (e / 8) % RC, j = e / (8 * RC);
                rec[j][rr][w] = (w < 7 && rr < rcn) ? src[((int64_t)(r0 + rr) * n + sid[j]) * 7 + w] : mk(0.f, 0.f);
            }
            __syncthreads();
            if (!active) continue;
#pragma unroll 2
            for (int j = sl; j < cnt; j += S) {
                const SrcHdr32 &q = hdr[j];
                const bool self = q.tri == ttri;
                const float dx = q.x - tx, dy = q.y - ty, dz = q.z - tz;
                if (CUT && dx * dx + dy * dy + dz * dz > rcut2) continue;   // damped below the cutoff
                const float R2 = self ? 1.f : dx * dx + dy * dy + dz * dz;
                const float iR = __builtin_amdgcn_rsqf(R2);
                const float R = R2 * iR;
                const float sn = __builtin_amdgcn_sinf(krev * R), cs = __builtin_amdgcn_cosf(krev * R);
                const float ex = LOSSY ? __builtin_amdgcn_exp2f(kexp * R) : 1.f;   // real k: no decay
                const float sc = self ? 0.f : inv4pi * iR * ex;            // e^{-Im k R} / (4 pi R)
                const cx<float> g = mk(sc * cs, sc * sn);                   // e^{ikR} / (4 pi R)
                const float iR2 = iR * iR;
                // f = (i k R - 1) g / R^2
                const cx<float> f = mk(iR2 * ((-ki * R - 1.f) * g.re - kr * R * g.im),
                                       iR2 * ((-ki * R - 1.f) * g.im + kr * R * g.re));
                const float v = q.nx * dx + q.ny * dy + q.nz * dz;
#pragma unroll
                for (int rr = 0; rr < RC; ++rr) {
                    const cx<float> *qr = rec[j][rr];
                    const cx<float> u = dx * qr[0] + dy * qr[1] + dz * qr[2];
                    const cx<float> wx = q.nx * u - v * qr[0] - dx * qr[6];
                    const cx<float> wy = q.ny * u - v * qr[1] - dy * qr[6];
                    const cx<float> wz = q.nz * u - v * qr[2] - dz * qr[6];
                    acc[rr][0] += f * wx + g * qr[3];
                    acc[rr][1] += f * wy + g * qr[4];
                    acc[rr][2] += f * wz + g * qr[5];
                }
            }
        }
        // sum the source slices, one right-hand side at a time
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) {
            __syncthreads();
            for (int c = 0; c < 3; ++c) red[threadIdx.x][c] = acc[rr][c];
            __syncthreads();
            if (threadIdx.x < ntc && rr < rcn) {
                cx<float> s[3] = {mk(0.f, 0.f), mk(0.f, 0.f), mk(0.f, 0.f)};
                for (int q = 0; q < S; ++q)
                    for (int c = 0; c < 3; ++c) s[c] += red[q * ntc + threadIdx.x][c];
                cx<float> *o = ys + ((int64_t)(r0 + rr) * n + t0 + tc0 + threadIdx.x) * 3;
                for (int c = 0; c < 3; ++c) o[c] += s[c];
            }
        }
    }
}

// local-only lossy plans: pairs beyond the cutoff radius are skipped by a branch
template <int RC>
constexpr auto k_p2p32_cut = k_p2p32<true, RC, true>;

// The near fields of the two plans of one BEM application at once, when the interior
// plan is local only (same nodes and octree; k0 real, k1 strongly lossy; one
// right-hand side per block row): the pair geometry, the LDS staging of the source
// headers and the reciprocal square root are shared, and each pair adds k0's terms
// and, within k1's cutoff radius, k1's.  Same layout and reduction as k_p2p32.
__global__ void __launch_bounds__(TPB) k_p2p32_pair(int nleaf, int nrhs, const int32_t *__restrict__ start,
                                                    const int32_t *__restrict__ nbr,
                                                    const double *__restrict__ center,
                                                    const double *__restrict__ spts, const double *__restrict__ snrm,
                                                    const int32_t *__restrict__ stri,
                                                    const cx<float> *__restrict__ src0,
                                                    const cx<float> *__restrict__ src1, int64_t n, double k0,
                                                    double k1_re, double k1_im, float rcut2_1,
                                                    cx<float> *__restrict__ ys0, cx<float> *__restrict__ ys1) {
    constexpr int TS = 128;
    __shared__ SrcHdr32 hdr[TS];
    __shared__ __attribute__((aligned(16))) cx<float> rec[2][TS][8];   // a[3], b[3], n.a, unused per plan
    __shared__ int32_t sid[TS];
    __shared__ int32_t nb_start[28], nb_box[27];
    __shared__ int n_nb;
    __shared__ cx<float> red[TPB][3];
    const int box = blockIdx.x, r = blockIdx.y;
    if (box >= nleaf || r >= nrhs) return;
    const int t0 = start[box], t1 = start[box + 1];
    const int nt = t1 - t0;
    const double c0x = center[3 * box], c0y = center[3 * box + 1], c0z = center[3 * box + 2];
    if (threadIdx.x == 0) {
        int c = 0, tot = 0;
        for (int q = 0; q < 27; ++q) {
            const int b = nbr[box * 27 + q];
            if (b >= 0) {
                nb_box[c] = b;
                nb_start[c] = tot;
                tot += start[b + 1] - start[b];
                ++c;
            }
        }
        nb_start[c] = tot;
        n_nb = c;
    }
    __syncthreads();
    const int ns_total = nb_start[n_nb];
    const float krev0 = (float)(k0 * 0.15915494309189533577), kr0 = (float)k0;
    const float krev1 = (float)(k1_re * 0.15915494309189533577);
    const float kexp1 = (float)(-k1_im * 1.44269504088896340736);
    const float kr1 = (float)k1_re, ki1 = (float)k1_im;
    const float inv4pi = 0.07957747154594766788f;
    for (int tc0 = 0; tc0 < nt; tc0 += TPB) {
        const int ntc = min(TPB, nt - tc0);
        const int S = TPB / ntc;
        const int ti = threadIdx.x % ntc, sl = threadIdx.x / ntc;
        const bool active = sl < S;
        const int64_t ig = t0 + tc0 + ti;
        float tx = 0.f, ty = 0.f, tz = 0.f;
        int32_t ttri = -1;
        if (active) {
            tx = (float)(spts[3 * ig] - c0x);
            ty = (float)(spts[3 * ig + 1] - c0y);
            tz = (float)(spts[3 * ig + 2] - c0z);
            ttri = stri[ig];
        }
        cx<float> acc0[3] = {mk(0.f, 0.f), mk(0.f, 0.f), mk(0.f, 0.f)};
        cx<float> acc1[3] = {mk(0.f, 0.f), mk(0.f, 0.f), mk(0.f, 0.f)};
        for (int base = 0; base < ns_total; base += TS) {
            const int cnt = min(TS, ns_total - base);
            __syncthreads();
            for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
                const int u = base + j;
                int b = 0;
                while (nb_start[b + 1] <= u) ++b;
                const int64_t sidx = start[nb_box[b]] + (u - nb_start[b]);
                SrcHdr32 q;
                q.x = (float)(spts[3 * sidx] - c0x);
                q.y = (float)(spts[3 * sidx + 1] - c0y);
                q.z = (float)(spts[3 * sidx + 2] - c0z);
                q.tri = stri[sidx];
                q.nx = (float)snrm[3 * sidx];
                q.ny = (float)snrm[3 * sidx + 1];
                q.nz = (float)snrm[3 * sidx + 2];
                q.pad = 0.f;
                hdr[j] = q;
                sid[j] = (int32_t)sidx;
            }
            __syncthreads();
            for (int e = threadIdx.x; e < cnt * 16; e += blockDim.x) {
                const int w = e % 8, pl = (e / 8) % 2, j = e / 16;
                const cx<float> *sp = pl ? src1 : src0;
                rec[pl][j][w] = w < 7 ? sp[((int64_t)r * n + sid[j]) * 7 + w] : mk(0.f, 0.f);
            }
            __syncthreads();
            if (!active) continue;
            for (int j = sl; j < cnt; j += S) {
                const SrcHdr32 &q = hdr[j];
                const bool self = q.tri == ttri;
                const float dx = q.x - tx, dy = q.y - ty, dz = q.z - tz;
                const float R2r = dx * dx + dy * dy + dz * dz;
                const float R2 = self ? 1.f : R2r;
                const float iR = __builtin_amdgcn_rsqf(R2);
                const float R = R2 * iR;
                const float iR2 = iR * iR;
                const float v = q.nx * dx + q.ny * dy + q.nz * dz;
                {
                    // k0 (real): g = e^{i k0 R} / (4 pi R), f = (i k0 R - 1) g / R^2
                    const float sn = __builtin_amdgcn_sinf(krev0 * R), cs = __builtin_amdgcn_cosf(krev0 * R);
                    const float sc = self ? 0.f : inv4pi * iR;
                    const cx<float> g = mk(sc * cs, sc * sn);
                    const cx<float> f = mk(iR2 * (-g.re - kr0 * R * g.im), iR2 * (-g.im + kr0 * R * g.re));
                    const cx<float> *qr = rec[0][j];
                    const cx<float> u = dx * qr[0] + dy * qr[1] + dz * qr[2];
                    const cx<float> wx = q.nx * u - v * qr[0] - dx * qr[6];
                    const cx<float> wy = q.ny * u - v * qr[1] - dy * qr[6];
                    const cx<float> wz = q.nz * u - v * qr[2] - dz * qr[6];
                    acc0[0] += f * wx + g * qr[3];
                    acc0[1] += f * wy + g * qr[4];
                    acc0[2] += f * wz + g * qr[5];
                }
                if (R2r <= rcut2_1) {
                    // k1 (lossy): the same with the decay e^{-Im k1 R}
                    const float sn = __builtin_amdgcn_sinf(krev1 * R), cs = __builtin_amdgcn_cosf(krev1 * R);
                    const float ex = __builtin_amdgcn_exp2f(kexp1 * R);
                    const float sc = self ? 0.f : inv4pi * iR * ex;
                    const cx<float> g = mk(sc * cs, sc * sn);
                    const cx<float> f = mk(iR2 * ((-ki1 * R - 1.f) * g.re - kr1 * R * g.im),
                                           iR2 * ((-ki1 * R - 1.f) * g.im + kr1 * R * g.re));
                    const cx<float> *qr = rec[1][j];
                    const cx<float> u = dx * qr[0] + dy * qr[1] + dz * qr[2];
                    const cx<float> wx = q.nx * u - v * qr[0] - dx * qr[6];
                    const cx<float> wy = q.ny * u - v * qr[1] - dy * qr[6];
                    const cx<float> wz = q.nz * u - v * qr[2] - dz * qr[6];
                    acc1[0] += f * wx + g * qr[3];
                    acc1[1] += f * wy + g * qr[4];
                    acc1[2] += f * wz + g * qr[5];
                }
            }
        }
        // sum the source slices, one plan at a time
        for (int pl = 0; pl < 2; ++pl) {
            __syncthreads();
            for (int c = 0; c < 3; ++c) red[threadIdx.x][c] = pl ? acc1[c] : acc0[c];
            __syncthreads();
            if (threadIdx.x < ntc) {
                cx<float> sm[3] = {mk(0.f, 0.f), mk(0.f, 0.f), mk(0.f, 0.f)};
                for (int q = 0; q < S; ++q)
                    for (int c = 0; c < 3; ++c) sm[c] += red[q * ntc + threadIdx.x][c];
                cx<float> *o = (pl ? ys1 : ys0) + ((int64_t)r * n + t0 + tc0 + threadIdx.x) * 3;
                for (int c = 0; c < 3; ++c) o[c] += sm[c];
            }
        }
    }
}

template <typename T>
__global__ void k_zero(cx<T> *__restrict__ x, int64_t m) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) x[i] = mk(T(0), T(0));
}

// ---------------------------------------------------------------- translations
// Batched GEMM grouped by operator: for every entry e of a tile,
//   Y[dst(e)] = T_op * X[src(e)]
// with X, Y column blocks of 3*nrhs columns of P2 complex coefficients.  The
// complex product is done as a real one: a complex column is read as its
// 2*P2 interleaved (re, im) reals and the operator is stored as the real
// 2P2 x 2P2 matrix with 2x2 blocks [[re, -im], [im, re]].  Each 64x64 block
// tile of the real product is computed by four waves of 16x16x4 MFMA
// instructions with operands staged through LDS.
struct Tile {
    int32_t op, first, count;
};
constexpr int TM = 64, TN = 64, TK = 16;
constexpr int OS_MAXCOLS = 288;                 // columns per operator-stationary job


template <typename T>
struct Mfma;
// Operand layout (both types): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16].
// Result layout differs: register q of lane l holds D[row][l % 16] with
//   f64 16x16x4: row = l / 16 + 4 q        f32 16x16x4: row = 4 (l / 16) + q
// (both checked with an on-device probe).
template <>
struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 mma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int q) { return (lane >> 4) + 4 * q; }
};
template <>
struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    __device__ static v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    __device__ static int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};

// Large operators (KR > 128 rows in FP64, > 256 in FP32): block tile of
// BG_M = 128 rows x big_n<T>() columns (64 in FP64, 128 in FP32), four waves in a
// 2 x 2 arrangement, each holding 4 x (big_n / 32) MFMA tiles.  K advances BG_K = 16 at a time; the next
// stage's A and B elements are fetched into registers while the MFMAs run on
// the current LDS buffer, then stored into the other buffer (one barrier per
// stage).  A is kept row-major in LDS (pitch BG_K + 1), B k-major (pitch
// BG_N + 1), so fragment reads and the transposing stores avoid bank conflicts.
constexpr int BG_M = 128, BG_K = 16;
// block columns: 64 in FP64 (keeps two waves per SIMD), 128 in FP32
template <typename T>
constexpr int big_n() { return sizeof(T) == 8 ? 64 : 128; }

template <typename T, bool ACCUM>
__global__ void __launch_bounds__(TPB) k_translate_big(const Tile *__restrict__ tiles, int ntiles,
                                                       const int32_t *__restrict__ ent,
                                                       const int32_t *__restrict__ src_map,
                                                       const T *__restrict__ ops, const T *__restrict__ X,
                                                       T *__restrict__ Y, int KR, int ncol, int64_t blkR) {
    typedef typename Mfma<T>::v4 v4;
    constexpr int BG_N = big_n<T>(), NJ = BG_N / 32;          // 16-column MFMA tiles per wave
    constexpr int AP = BG_K + 1, BP = BG_N + 1;
    constexpr int LA = BG_M * BG_K / TPB, LB = BG_K * BG_N / TPB;   // elements per thread and stage
    __shared__ T As[2][BG_M * AP];
    __shared__ T Bs[2][BG_K * BP];
    __shared__ int64_t s_in[BG_N], s_out[BG_N];
    const int tix = xcd_tile(blockIdx.x, ntiles);
    if (tix >= ntiles) return;
    const Tile tl = tiles[tix];
    const int r0 = blockIdx.y * BG_M;
    const T *Top = ops + (size_t)tl.op * KR * KR;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wr0 = (wave >> 1) * 64, wc0 = (wave & 1) * (BG_N / 2);
    const int Ctot = tl.count * ncol;
    const int nk = (KR + BG_K - 1) / BG_K;
    T pa[LA], pb[LB];
    for (int c0 = 0; c0 < Ctot; c0 += BG_N) {
        const int C = min(BG_N, Ctot - c0);
        __syncthreads();                                  // s_in/s_out and LDS buffers of the previous chunk
        for (int c = threadIdx.x; c < BG_N; c += blockDim.x) {
            if (c < C) {
                const int cg = c0 + c;
                const int e = cg / ncol, cc = cg % ncol;
                const int32_t en = ent[tl.first + e];
                const int32_t sb = src_map ? src_map[en] : en;
                s_in[c] = (int64_t)sb * blkR + (int64_t)cc * KR;
                s_out[c] = (int64_t)en * blkR + (int64_t)cc * KR;
            } else {
                s_in[c] = -1;
                s_out[c] = -1;
            }
        }
        __syncthreads();
        auto fetch = [&](int ks) {
            const int k0 = ks * BG_K;
#pragma unroll
            for (int j = 0; j < LA; ++j) {
                const int idx = threadIdx.x + j * TPB;
                const int r = idx / BG_K, kk = idx % BG_K;
                pa[j] = (r0 + r < KR && k0 + kk < KR) ? Top[(size_t)(r0 + r) * KR + k0 + kk] : T(0);
            }
#pragma unroll
            for (int j = 0; j < LB; ++j) {
                const int idx = threadIdx.x + j * TPB;
                const int c = idx / BG_K, kk = idx % BG_K;
                const int64_t o = s_in[c];
                pb[j] = (o >= 0 && k0 + kk < KR) ? X[o + k0 + kk] : T(0);
            }
        };
        auto stash = [&](int buf) {
#pragma unroll
            for (int j = 0; j < LA; ++j) {
                const int idx = threadIdx.x + j * TPB;
                As[buf][(idx / BG_K) * AP + idx % BG_K] = pa[j];
            }
#pragma unroll
            for (int j = 0; j < LB; ++j) {
                const int idx = threadIdx.x + j * TPB;
                Bs[buf][(idx % BG_K) * BP + idx / BG_K] = pb[j];
            }
        };
        v4 acc[4][NJ];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[i][j] = v4{0, 0, 0, 0};
        fetch(0);
        stash(0);
        __syncthreads();
        for (int ks = 0; ks < nk; ++ks) {
            const int buf = ks & 1;
            if (ks + 1 < nk) fetch(ks + 1);
            const T *A = As[buf], *B = Bs[buf];
#pragma unroll
            for (int k4 = 0; k4 < BG_K; k4 += 4) {
                T a[4], b[NJ];
#pragma unroll
                for (int i = 0; i < 4; ++i) a[i] = A[(wr0 + 16 * i + (lane & 15)) * AP + k4 + (lane >> 4)];
#pragma unroll
                for (int j = 0; j < NJ; ++j) b[j] = B[(k4 + (lane >> 4)) * BP + wc0 + 16 * j + (lane & 15)];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j) acc[i][j] = Mfma<T>::mma(a[i], b[j], acc[i][j]);
            }
            if (ks + 1 < nk) stash(buf ^ 1);
            __syncthreads();
        }
        // ACCUM is a template parameter: the overwrite instance carries no loads of Y
        if (ACCUM) {
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int col = wc0 + 16 * j + (lane & 15);
                if (col >= C) continue;
                T *yo = Y + s_out[col];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int row = r0 + wr0 + 16 * i + Mfma<T>::row(lane, q);
                        if (row < KR) yo[row] += acc[i][j][q];
                    }
            }
        } else {
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const int col = wc0 + 16 * j + (lane & 15);
                if (col >= C) continue;
                T *yo = Y + s_out[col];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int row = r0 + wr0 + 16 * i + Mfma<T>::row(lane, q);
                        if (row < KR) yo[row] = acc[i][j][q];
                    }
            }
        }
    }
}


// Variant for small operators (2 p^2 <= 16 RT): every block computes all rows
// of its 64 columns, so each gathered column is read from memory once.  The
// four waves split the columns (16 each); every wave holds RT 16x16 tiles.
template <typename T, int RT>
__global__ void __launch_bounds__(TPB) k_translate_fm(const Tile *__restrict__ tiles, int ntiles,
                                                      const int32_t *__restrict__ ent,
                                                      const int32_t *__restrict__ src_map, const T *__restrict__ ops,
                                                      const T *__restrict__ X, T *__restrict__ Y, int KR, int ncol,
                                                      int64_t blkR, int accum) {
    typedef typename Mfma<T>::v4 v4;
    __shared__ T As[RT * 16][TK + 1];
    __shared__ T Bs[TK][TN];
    __shared__ int32_t s_src[TN], s_dst[TN];
    const int tix = xcd_tile(blockIdx.x, ntiles);
    if (tix >= ntiles) return;
    const Tile tl = tiles[tix];
    const T *Top = ops + (size_t)tl.op * KR * KR;
    for (int q = threadIdx.x; q < tl.count && q < TN; q += blockDim.x) {
        int32_t e = ent[tl.first + q];
        s_dst[q] = e;
        s_src[q] = src_map ? src_map[e] : e;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wc0 = wave * 16;
    const int Ctot = tl.count * ncol;
    for (int c0 = 0; c0 < Ctot; c0 += TN) {
        const int C = min(TN, Ctot - c0);
        v4 acc[RT];
#pragma unroll
        for (int i = 0; i < RT; ++i) acc[i] = v4{0, 0, 0, 0};
        for (int k0 = 0; k0 < KR; k0 += TK) {
            __syncthreads();
            for (int t = threadIdx.x; t < RT * 16 * TK; t += blockDim.x) {
                const int rr = t / TK, kk = t % TK;
                As[rr][kk] = (rr < KR && k0 + kk < KR) ? Top[(size_t)rr * KR + k0 + kk] : T(0);
            }
            for (int t = threadIdx.x; t < TN * TK; t += blockDim.x) {
                const int c = t / TK, kk = t % TK;
                T v = T(0);
                if (c < C && k0 + kk < KR) {
                    const int cg = c0 + c;
                    const int e = cg / ncol, cc = cg % ncol;
                    v = X[(int64_t)s_src[e] * blkR + (int64_t)cc * KR + k0 + kk];
                }
                Bs[kk][c] = v;
            }
            __syncthreads();
#pragma unroll
            for (int k4 = 0; k4 < TK; k4 += 4) {
                const T b = Bs[k4 + (lane >> 4)][wc0 + (lane & 15)];
#pragma unroll
                for (int i = 0; i < RT; ++i) {
                    const T a = As[16 * i + (lane & 15)][k4 + (lane >> 4)];
                    acc[i] = Mfma<T>::mma(a, b, acc[i]);
                }
            }
        }
        const int col = wc0 + (lane & 15);
        if (col < C) {
            const int cg = c0 + col;
            const int e = cg / ncol, cc = cg % ncol;
            T *yo = Y + (int64_t)s_dst[e] * blkR + (int64_t)cc * KR;
#pragma unroll
            for (int i = 0; i < RT; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = 16 * i + Mfma<T>::row(lane, q);
                    if (row < KR) yo[row] = accum ? yo[row] + acc[i][q] : acc[i][q];
                }
        }
    }
}

// Operator-stationary variant for FP32 operators with 2 p^2 <= 164 (p <= 9):
// a block owns one operator and a long run of that operator's columns.  Each
// of its four waves loads the MFMA A-fragments of its RTW row tiles for the
// whole K extent into registers once (a[i][kk] = T[16 i + l%16][4 kk + l/16]),
// then the block streams the columns 16 at a time through double-buffered LDS.
// Operator traffic drops from one read per 64 columns to one read per job.
constexpr int OS_COLS = 16;

template <int KS, int RTW>
__global__ void __launch_bounds__(TPB) k_translate_os(const Tile *__restrict__ tiles, int ntiles,
                                                      const int32_t *__restrict__ ent,
                                                      const int32_t *__restrict__ src_map,
                                                      const float *__restrict__ ops, const float *__restrict__ X,
                                                      float *__restrict__ Y, int KR, int ncol, int64_t blkR, int accum) {
    constexpr int KP = KS * 4;                     // K padded to whole MFMA k-steps
    constexpr int LD = (KP * OS_COLS + TPB - 1) / TPB;
    typedef typename Mfma<float>::v4 v4;
    __shared__ float Bs[2][KP][OS_COLS];
    __shared__ int64_t s_in[OS_MAXCOLS], s_out[OS_MAXCOLS];
    const int tix = xcd_tile(blockIdx.x, ntiles);
    if (tix >= ntiles) return;
    const Tile tl = tiles[tix];
    const int C = tl.count * ncol;                 // <= OS_MAXCOLS (plan-time tiling)
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        const int e = c / ncol, cc = c % ncol;
        const int32_t en = ent[tl.first + e];
        const int32_t sb = src_map ? src_map[en] : en;
        s_in[c] = (int64_t)sb * blkR + (int64_t)cc * KR;
        s_out[c] = (int64_t)en * blkR + (int64_t)cc * KR;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float *Top = ops + (size_t)tl.op * KR * KR;
    float a[RTW][KS];
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
        const int row = (wave * RTW + i) * 16 + (lane & 15);
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const int k = 4 * kk + (lane >> 4);
            a[i][kk] = (row < KR && k < KR) ? Top[(size_t)row * KR + k] : 0.f;
        }
    }
    __syncthreads();
    const int ntc = (C + OS_COLS - 1) / OS_COLS;
    float pre[LD];
    auto fetch = [&](int t) {
#pragma unroll
        for (int j = 0; j < LD; ++j) {
            const int e = threadIdx.x + j * TPB;
            const int c = e / KP, k = e % KP;
            const int cg = t * OS_COLS + c;
            pre[j] = (e < KP * OS_COLS && cg < C && k < KR) ? X[s_in[cg] + k] : 0.f;
        }
    };
    auto stash = [&](int buf) {
#pragma unroll
        for (int j = 0; j < LD; ++j) {
            const int e = threadIdx.x + j * TPB;
            if (e < KP * OS_COLS) Bs[buf][e % KP][e / KP] = pre[j];
        }
    };
    fetch(0);
    stash(0);
    __syncthreads();
    for (int t = 0; t < ntc; ++t) {
        const int buf = t & 1;
        if (t + 1 < ntc) fetch(t + 1);
        v4 acc[RTW];
#pragma unroll
        for (int i = 0; i < RTW; ++i) acc[i] = v4{0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < KS; ++kk) {
            const float b = Bs[buf][4 * kk + (lane >> 4)][lane & 15];
#pragma unroll
            for (int i = 0; i < RTW; ++i) acc[i] = Mfma<float>::mma(a[i][kk], b, acc[i]);
        }
        const int cg = t * OS_COLS + (lane & 15);
        if (cg < C) {
            float *yo = Y + s_out[cg];
#pragma unroll
            for (int i = 0; i < RTW; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = (wave * RTW + i) * 16 + Mfma<float>::row(lane, q);
                    if (row < KR) yo[row] = accum ? yo[row] + acc[i][q] : acc[i][q];
                }
        }
        if (t + 1 < ntc) stash(buf ^ 1);
        __syncthreads();
    }
}

// operators with more than 128 (FP64) or 256 (FP32) real rows take k_translate_big
inline bool use_big(int precision, int KR) {
    const int rt = (KR + 15) / 16;
    return !(rt <= 16 && (precision == FMB_FP32 || rt <= 8));
}

// columns per split-BF16 job (the instantiations in launch_translate)
inline int bf3_job_cols(int p) { return p <= 5 ? 96 : (p <= 8 ? 64 : 32); }

inline bool use_bf3(const Plan &P) {
    return P.precision == FMB_FP32 && P.translate_mode == FMB_TRANSLATE_BF16X3 && P.order >= 2 && P.order <= 9;
}

// the operator-stationary kernel applies to FP32 operators of order 2 <= p <= 9
inline bool use_os(int precision, int p, int nrhs_max) {
    (void)nrhs_max;
    return precision == FMB_FP32 && p >= 2 && p <= 9;
}

// right-hand sides per translation launch: a job holds whole entries of 3 x (this many)
// columns, so wider batches run as several launches over slices of the right-hand sides
inline int translate_rhs_chunk(const Plan &P) {
    if (use_bf3(P)) return std::min(P.nrhs_max, bf3_job_cols(P.order) / 3);
    if (use_os(P.precision, P.order, P.nrhs_max)) return std::min(P.nrhs_max, OS_MAXCOLS / 3);
    return P.nrhs_max;
}

// Split-BF16 variant of the operator-stationary kernel (FP32 plans, p <= 9).
// x = hi + lo with hi = bf16(x), lo = bf16(x - hi); a product is taken as
// a_hi b_hi + a_hi b_lo + a_lo b_hi on the 16x16x32 BF16 MFMA with FP32
// accumulation (the lo*lo term, ~2^-16 relative, is dropped).  Operators are
// pre-split at plan time and stored fragment-major: lane l of row tile i and
// k-step s holds T[16 i + l%16][32 s + 8 (l/16) + j], j = 0..7.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// A job holds at most JC columns (bf3_job_cols); all of them are staged into
// LDS with one batch of loads before any MFMA runs, so a job waits for memory
// once instead of once per 16-column chunk.
// ROLE only names the launch in kernel traces: 0 S|S (M2M), 1 S|R (M2L), 2 R|R (L2L).
template <int KS, int RTW, int JC, int ROLE>
__global__ void __launch_bounds__(TPB) k_translate_bf3(const Tile *__restrict__ tiles, int ntiles,
                                                       const int32_t *__restrict__ ent,
                                                       const int32_t *__restrict__ src_map,
                                                       const bf16x8 *__restrict__ fhi,
                                                       const bf16x8 *__restrict__ flo, const float *__restrict__ X,
                                                       float *__restrict__ Y, int KR, int RT, int ncol,
                                                       int64_t blkR, int accum) {
    constexpr int KP = KS * 32;
    constexpr int CS = KP + 4;                                   // LDS column stride (floats)
    constexpr int LD = (KP * JC + TPB - 1) / TPB;
    typedef typename Mfma<float>::v4 v4;
    constexpr int RP = 64 * RTW + 1;                             // output tile pitch (rows of 4 waves)
    __shared__ __attribute__((aligned(16))) float Bs[JC][CS];
    __shared__ float Os[16][RP];
    __shared__ int64_t s_in[JC], s_out[JC];
    const int tix = xcd_tile(blockIdx.x, ntiles);
    if (tix >= ntiles) return;
    const Tile tl = tiles[tix];
    const int C = tl.count * ncol;                               // <= JC (plan-time tiling)
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
        const int e = c / ncol, cc = c % ncol;
        const int32_t en = ent[tl.first + e];
        const int32_t sb = src_map ? src_map[en] : en;
        s_in[c] = (int64_t)sb * blkR + (int64_t)cc * KR;
        s_out[c] = (int64_t)en * blkR + (int64_t)cc * KR;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    bf16x8 ah[RTW][KS], al[RTW][KS];
#pragma unroll
    for (int i = 0; i < RTW; ++i) {
        const int tile = wave * RTW + i;
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            if (tile < RT) {
                const size_t f = (((size_t)tl.op * RT + tile) * KS + s) * 64 + lane;
                ah[i][s] = fhi[f];
                al[i][s] = flo[f];
            } else {
                for (int j = 0; j < 8; ++j) {
                    ah[i][s][j] = (__bf16)0.f;
                    al[i][s][j] = (__bf16)0.f;
                }
            }
        }
    }
    __syncthreads();
    {
        float pre[LD];
#pragma unroll
        for (int j = 0; j < LD; ++j) {
            const int e = threadIdx.x + j * TPB;
            const int c = e / KP, k = e % KP;
            pre[j] = (e < KP * JC && c < C && k < KR) ? X[s_in[c] + k] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < LD; ++j) {
            const int e = threadIdx.x + j * TPB;
            if (e < KP * JC) Bs[e / KP][e % KP] = pre[j];
        }
    }
    __syncthreads();
    const int ntc = (C + 15) / 16;
    for (int t = 0; t < ntc; ++t) {
        v4 acc[RTW];
#pragma unroll
        for (int i = 0; i < RTW; ++i) acc[i] = v4{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const float *bp = &Bs[16 * t + (lane & 15)][32 * s + 8 * (lane >> 4)];
            const float4 v0 = *reinterpret_cast<const float4 *>(bp);
            const float4 v1 = *reinterpret_cast<const float4 *>(bp + 4);
            const float v[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
            bf16x8 bh, bl;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const __bf16 h = (__bf16)v[j];
                bh[j] = h;
                bl[j] = (__bf16)(v[j] - (float)h);
            }
#pragma unroll
            for (int i = 0; i < RTW; ++i) {
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i][s], bh, acc[i], 0, 0, 0);
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i][s], bl, acc[i], 0, 0, 0);
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i][s], bh, acc[i], 0, 0, 0);
            }
        }
        // the 16 x KR output tile goes through LDS so that every column is
        // written as one contiguous run of KR floats
#pragma unroll
        for (int i = 0; i < RTW; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) Os[lane & 15][(wave * RTW + i) * 16 + 4 * (lane >> 4) + q] = acc[i][q];
        __syncthreads();
        const int cn = min(16, C - 16 * t);
        for (int e = threadIdx.x; e < cn * KR; e += TPB) {
            const int c = e / KR, row = e % KR;
            float *yo = Y + s_out[16 * t + c] + row;
            *yo = accum ? *yo + Os[c][row] : Os[c][row];
        }
        __syncthreads();
    }
}

// plan-time split of FP32 operators into fragment-major BF16 hi/lo parts
__global__ void k_split_bf16(const float *__restrict__ T, int nops, int KR, int RT, int KS, bf16x8 *__restrict__ hi,
                             bf16x8 *__restrict__ lo) {
    const int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t total = (int64_t)nops * RT * KS * 64;
    if (f >= total) return;
    const int lane = (int)(f % 64);
    const int s = (int)((f / 64) % KS);
    const int tile = (int)((f / (64 * KS)) % RT);
    const int64_t op = f / ((int64_t)64 * KS * RT);
    const int row = 16 * tile + (lane & 15);
    bf16x8 h, l;
    for (int j = 0; j < 8; ++j) {
        const int k = 32 * s + 8 * (lane >> 4) + j;
        const float x = (row < KR && k < KR) ? T[((size_t)op * KR + row) * KR + k] : 0.f;
        const __bf16 xh = (__bf16)x;
        h[j] = xh;
        l[j] = (__bf16)(x - (float)xh);
    }
    hi[f] = h;
    lo[f] = l;
}

template <int ROLE>
void launch_bf3(int p, unsigned g, const Tile *tiles, int64_t ntiles, const int32_t *ent, const int32_t *src_map,
                const bf16x8 *h, const bf16x8 *l, const float *x, float *y, int KR, int RT, int ncol, int64_t blkR,
                int accum, hipStream_t s) {
    const int nt = (int)ntiles;
    switch (p) {
        case 2:
        case 3:
        case 4: k_translate_bf3<1, 1, 96, ROLE><<<g, TPB, 0, s>>>(tiles, nt, ent, src_map, h, l, x, y, KR, RT, ncol, blkR, accum); break;
        case 5: k_translate_bf3<2, 1, 96, ROLE><<<g, TPB, 0, s>>>(tiles, nt, ent, src_map, h, l, x, y, KR, RT, ncol, blkR, accum); break;
        case 6: k_translate_bf3<3, 2, 64, ROLE><<<g, TPB, 0, s>>>(tiles, nt, ent, src_map, h, l, x, y, KR, RT, ncol, blkR, accum); break;
        case 7:
        case 8: k_translate_bf3<4, 2, 64, ROLE><<<g, TPB, 0, s>>>(tiles, nt, ent, src_map, h, l, x, y, KR, RT, ncol, blkR, accum); break;
        default: k_translate_bf3<6, 3, 32, ROLE><<<g, TPB, 0, s>>>(tiles, nt, ent, src_map, h, l, x, y, KR, RT, ncol, blkR, accum); break;
    }
}

// role: 0 S|S, 1 S|R, 2 R|R (names the split-BF16 launches in kernel traces);
// accum: add the products into Y instead of overwriting it
template <typename T>
void launch_translate(const Tile *tiles, int64_t ntiles, const int32_t *ent, const int32_t *src_map, const T *ops,
                      const T *X, T *Y, int KR, int ncol, int64_t blkR, bool os, hipStream_t s, int role, int accum,
                      const void *fhi = nullptr, const void *flo = nullptr) {
    if (ntiles <= 0) return;
    if (fhi) {
        // split-BF16 translations (FP32 plans only, checked by use_bf3)
        const int p = (int)lround(sqrt(KR / 2.0));
        const int RT = (KR + 15) / 16;
        // register tiles per instantiation below: KS k-steps of 32, 4 waves x RTW row tiles of 16
        static const int ks_of[10] = {0, 0, 1, 1, 1, 2, 3, 4, 4, 6}, rtw_of[10] = {0, 0, 1, 1, 1, 1, 2, 2, 2, 3};
        if (p < 2 || p > 9 || 2 * p * p != KR || (KR + 31) / 32 != ks_of[p] || RT > 4 * rtw_of[p])
            throw std::runtime_error("split-BF16 translation: unsupported operator size");
        const unsigned g = (unsigned)(((ntiles + 7) / 8) * 8);
        const bf16x8 *h = (const bf16x8 *)fhi, *l = (const bf16x8 *)flo;
        const float *x = (const float *)X;
        float *y = (float *)Y;
        switch (role) {
            case 0: launch_bf3<0>(p, g, tiles, ntiles, ent, src_map, h, l, x, y, KR, RT, ncol, blkR, accum, s); break;
            case 1: launch_bf3<1>(p, g, tiles, ntiles, ent, src_map, h, l, x, y, KR, RT, ncol, blkR, accum, s); break;
            default: launch_bf3<2>(p, g, tiles, ntiles, ent, src_map, h, l, x, y, KR, RT, ncol, blkR, accum, s); break;
        }
        FMB_LAUNCH_CHECK();
        return;
    }
    const int rt = (KR + 15) / 16;
    const unsigned g = (unsigned)(((ntiles + 7) / 8) * 8);
    if (os) {
        const float *o = (const float *)ops;
        const float *x = (const float *)X;
        float *y = (float *)Y;
        const int p = (int)lround(sqrt(KR / 2.0));
        switch (p) {
            case 2: k_translate_os<2, 1><<<g, TPB, 0, s>>>(tiles, (int)ntiles, ent, src_map, o, x, y, KR, ncol, blkR, accum); break;
            case 3: k_translate_os<5, 1><<<g, TPB, 0, s>>>(tiles, (int)ntiles, ent, src_map, o, x, y, KR, ncol, blkR, accum); break;
            case 4: k_translate_os<8, 1><<<g, TPB, 0, s>>>(tiles, (int)ntiles, ent, src_map, o, x, y, KR, ncol, blkR, accum); break;
            case 5: k_translate_os<13, 1><<<g, TPB, 0, s>>>(tiles, (int)ntiles, ent, src_map, o, x, y, KR, ncol, blkR, accum); break;
            case 6: k_translate_os<18, 2><<<g, TPB, 0, s>>>(tiles, (int)ntiles, ent, src_map, o, x, y, KR, ncol, blkR, accum); break;
            case 7: k_translate_os<25, 2><<<g, TPB, 0, s>>>(tiles, (int)ntiles, ent, src_map, o, x, y, KR, ncol, blkR, accum); break;
            case 8: k_translate_os<32, 2><<<g, TPB, 0, s>>>(tiles, (int)ntiles, ent, src_map, o, x, y, KR, ncol, blkR, accum); break;
            default: k_translate_os<41, 3><<<g, TPB, 0, s>>>(tiles, (int)ntiles, ent, src_map, o, x, y, KR, ncol, blkR, accum); break;
        }
        FMB_LAUNCH_CHECK();
        return;
    }
#define FMB_FM(R)                                                                                                   \
    case R:                                                                                                         \
        k_translate_fm<T, R><<<g, TPB, 0, s>>>(tiles, (int)ntiles, ent, src_map, ops, X, Y, KR, ncol, blkR, accum); \
        break;
    if (!use_big(sizeof(T) == 4 ? FMB_FP32 : FMB_FP64, KR)) {
        switch (rt) {
            FMB_FM(1) FMB_FM(2) FMB_FM(3) FMB_FM(4) FMB_FM(5) FMB_FM(6) FMB_FM(7) FMB_FM(8)
            FMB_FM(9) FMB_FM(10) FMB_FM(11) FMB_FM(12) FMB_FM(13) FMB_FM(14) FMB_FM(15) FMB_FM(16)
            default: break;
        }
    } else {
        const unsigned rowblocks = (unsigned)((KR + BG_M - 1) / BG_M);
        if (accum)
            k_translate_big<T, true><<<dim3(g, rowblocks), TPB, 0, s>>>(tiles, (int)ntiles, ent, src_map, ops, X, Y, KR,
                                                                        ncol, blkR);
        else
            k_translate_big<T, false><<<dim3(g, rowblocks), TPB, 0, s>>>(tiles, (int)ntiles, ent, src_map, ops, X, Y,
                                                                         KR, ncol, blkR);
    }
#undef FMB_FM
    FMB_LAUNCH_CHECK();
}

// parent (level l) multipole = sum of its children's translated slots
// Column sums of a row range [e0, e1) of slots (rows of blk complex values, the
// first ncolP2 of which are used) by one block: columns go in chunks of
// CW = min(ncolP2, 128); within a chunk G = TPB / CW row groups take rows
// e0 + g, e0 + g + G, ... and their partial sums are added in group order, so
// the result does not depend on timing.
template <typename T>
__device__ inline void slot_sum(const cx<T> *__restrict__ Y, int e0, int e1, int64_t blk, int ncolP2,
                                cx<T> *__restrict__ out, bool accumulate, cx<T> *sm) {
    const int t = threadIdx.x;
    const int CW = min(ncolP2, 128), G = TPB / CW;
    const int g = t / CW, c = t % CW;
    for (int c0 = 0; c0 < ncolP2; c0 += CW) {
        const int cw = min(CW, ncolP2 - c0);
        cx<T> s = mk(T(0), T(0));
        if (g < G && c < cw) {
#pragma unroll 4
            for (int e = e0 + g; e < e1; e += G) s += Y[(int64_t)e * blk + c0 + c];
        }
        sm[t] = s;
        __syncthreads();
        if (t < cw) {
            cx<T> tot = sm[t];
            for (int q = 1; q < G; ++q) tot += sm[q * CW + t];
            if (accumulate) out[c0 + t] += tot;
            else out[c0 + t] = tot;
        }
        __syncthreads();
    }
}

// parent multipole = sum of its children's S|S slots
template <typename T>
__global__ void __launch_bounds__(TPB) k_sum_children(const int32_t *__restrict__ child_start, int64_t nbox,
                                                      const cx<T> *__restrict__ Yc, cx<T> *__restrict__ Mp, int64_t blk,
                                                      int ncolP2) {
    __shared__ cx<T> sm[TPB];
    const int64_t b = blockIdx.x;
    slot_sum(Yc, child_start[b], child_start[b + 1], blk, ncolP2, Mp + b * blk, false, sm);
}

// The S|R slot sums of every level in one launch: block b belongs to the level
// l with box0[l] <= b < box0[l + 1]; that level's box b - box0[l] sums its
// slots into its local expansion (overwriting it).
struct FarSumLevels {
    int nlev;
    int64_t box0[MAX_DEPTH + 2];
    const int32_t *ff_ofs[MAX_DEPTH + 1];
    int64_t slot_base[MAX_DEPTH + 1];
    void *L[MAX_DEPTH + 1];
};

template <typename T>
__global__ void __launch_bounds__(TPB) k_sum_far_all(FarSumLevels lv, const cx<T> *__restrict__ Yf, int64_t blk,
                                                     int ncolP2) {
    __shared__ cx<T> sm[TPB];
    const int64_t gb = blockIdx.x;
    int l = 0;
    while (l + 1 < lv.nlev && lv.box0[l + 1] <= gb) ++l;
    const int64_t b = gb - lv.box0[l];
    const int32_t *ofs = lv.ff_ofs[l];
    slot_sum(Yf + lv.slot_base[l] * blk, ofs[b], ofs[b + 1], blk, ncolP2, (cx<T> *)lv.L[l] + b * blk, false, sm);
}

inline unsigned gridn(int64_t m, int tpb = TPB) { return (unsigned)((m + tpb - 1) / tpb); }

// One product is a fixed sequence of steps (a launch or a short run of
// launches); matvec_step issues step number `step` and returns false past the
// last one, so that two products on two streams can be issued alternately.
template <typename T>
bool matvec_step(Plan &P, const cx<T> *a, const cx<T> *b, cx<T> *y, int nrhs, hipStream_t s, int step) {
    const int64_t n = P.n;
    const int L = P.depth, p = P.order, P2 = P.P2;
    const int64_t blk = (int64_t)P.nrhs_max * 3 * P2;
    const int ncol = 3 * nrhs;
    const int KR = 2 * P2;                          // real rows of the embedded operators
    const int64_t blkR = 2 * blk;
    const bool os = use_os(P.precision, p, P.nrhs_max);
    const bool bf3 = use_bf3(P);
    // translations run over slices of at most cw right-hand sides; roff(r0) is the
    // offset (in reals) of right-hand side r0 inside a box's or slot's block
    const int cw = translate_rhs_chunk(P);
    auto roff = [&](int r0) { return (int64_t)r0 * 3 * KR; };
    cx<T> *src = P.src.as<cx<T>>();
    cx<T> *ys = P.ys.as<cx<T>>();
    cx<T> *yb = P.ybuf.as<cx<T>>();
    StageTimer &tm = P.timer;
    hipEvent_t ev = nullptr;
    int k = 0;
    if (step == k++) {
        tm.begin(ST_GATHER, s, ev);
        k_gather_src<T><<<gridn(n), TPB, 0, s>>>(a, b, P.perm.as<int32_t>(), P.sw.as<double>(), P.snrm.as<double>(), n,
                                                 nrhs, src);
        FMB_LAUNCH_CHECK();
        tm.end(ST_GATHER, s, ev);
        return true;
    }
    // Step 1: leaf multipoles
    Level &LL = P.lv[L];
    const bool far = P.far_on();
    const int lmin = std::max(2, P.far_lmin);
    if (step == k++) {
        if (!far) return true;
        const int N = p;
        const size_t per = ((size_t)(N + 1) * (N + 2) + 1 + 7) * sizeof(cx<T>) + 6 * sizeof(T);
        // LDS: the group-reduction area (G * P2 * 3 complex when G > 1), then per node of a batch
        const int G = P2 <= TPB ? TPB / P2 : 1;
        const size_t redb = G > 1 ? (size_t)G * P2 * 3 * sizeof(cx<T>) : 0;
        // node batches sized so that the block's LDS stays near 24 KB (several blocks share a CU), with at
        // least 8 nodes per batch while 60 KB allow it
        const size_t fit = (60000 - redb) / per;
        const size_t want = std::max<size_t>(8, (redb < 24000 ? 24000 - redb : 0) / per);
        const int batch = (int)std::max<size_t>(1, std::min<size_t>({(size_t)64, fit, want}));
        const size_t sh = redb + (size_t)batch * per;
        FMB_REQUIRE(P2 <= P2M_SLOTS_MAX * TPB, "leaf order too large for the multipole kernel");
        auto kern = P2 <= P2M_SLOTS * TPB ? k_p2m<T, P2M_SLOTS> : k_p2m<T, P2M_SLOTS_MAX>;
        tm.begin(ST_P2M, s, ev);
        kern<<<(unsigned)LL.nbox, TPB, sh, s>>>(
            LL.start.as<int32_t>(), LL.center.as<double>(), P.spts.as<double>(), P.snrm.as<double>(), src, n, p, P.k_re,
            P.k_im, P.inv_alpha.as<double>() + (size_t)L * p, P.btab.as<T>(), P.bgix.as<int32_t>(), nrhs, P.nrhs_max,
            batch, LL.M.as<cx<T>>());
        FMB_LAUNCH_CHECK();
        tm.end(ST_P2M, s, ev);
        return true;
    }
    // Step 2: upward pass (S|S), levels L-1 .. 2
    for (int l = L - 1; l >= 2; --l) {
        Level &V = P.lv[l], &C = P.lv[l + 1];
        if (step != k++) continue;
        if (l < lmin) return true;
        if (P.hf) {
            tm.begin(ST_M2M, s, ev);
            hf_m2m<T>(P, l, nrhs, s);
            tm.end(ST_M2M, s, ev);
            return true;
        }
        if (V.ntiles_m2m == 0) return true;
        tm.begin(ST_M2M, s, ev);
        for (int r0 = 0; r0 < nrhs; r0 += cw)
            launch_translate<T>(V.tiles_m2m.as<Tile>(), V.ntiles_m2m, C.by_octant.as<int32_t>(), nullptr, V.m2m.as<T>(),
                                (const T *)C.M.p + roff(r0), (T *)yb + roff(r0), KR, 3 * std::min(cw, nrhs - r0), blkR,
                                os, s, 0, 0, bf3 ? V.m2m_hi.p : nullptr, V.m2m_lo.p);
        tm.end(ST_M2M, s, ev, (nrhs + cw - 1) / cw);
        tm.begin(ST_SUMS, s, ev);
        k_sum_children<T><<<(unsigned)V.nbox, TPB, 0, s>>>(V.child_start.as<int32_t>(), V.nbox, yb, V.M.as<cx<T>>(), blk,
                                                           ncol * P2);
        FMB_LAUNCH_CHECK();
        tm.end(ST_SUMS, s, ev);
        return true;
    }
    // Step 3a: S|R of every level, one run of launches; each level's slots have
    // their own region of the slot buffer (slot_base)
    if (step == k++) {
        if (!far) return true;
        int nk = 0;
        tm.begin(ST_M2L, s, ev);
        if (P.hf) {
            // each target sums its own far-field translations and writes its local expansion
            for (int l = lmin; l < L; ++l) hf_m2l<T>(P, l, nrhs, s);
            hipEvent_t ev2 = nullptr;
            tm.begin(ST_M2L_FINE, s, ev2);
            hf_m2l<T>(P, L, nrhs, s);
            tm.end(ST_M2L_FINE, s, ev2, 1);
            tm.end(ST_M2L, s, ev, L - lmin + 1);
            return true;
        }
        for (int l = lmin; l <= L; ++l) {
            Level &V = P.lv[l];
            if (V.ntiles_m2l == 0) continue;
            for (int r0 = 0; r0 < nrhs; r0 += cw) {
                launch_translate<T>(V.tiles_m2l.as<Tile>(), V.ntiles_m2l, V.ff_by_op.as<int32_t>(),
                                    V.ff_src.as<int32_t>(), V.m2l.as<T>(), (const T *)V.M.p + roff(r0),
                                    (T *)(yb + V.slot_base * blk) + roff(r0), KR, 3 * std::min(cw, nrhs - r0), blkR,
                                    os, s, 1, 0, bf3 ? V.m2l_hi.p : nullptr, V.m2l_lo.p);
                ++nk;
            }
        }
        tm.end(ST_M2L, s, ev, nk);
        return true;
    }
    // Step 3b: the S|R slot sums of every level (one launch, overwriting L),
    // then R|R from the parent added into each level in turn
    if (step == k++) {
        if (!far || P.hf) return true;
        FarSumLevels fs{};
        fs.nlev = L - lmin + 1;
        int64_t tot = 0;
        for (int l = lmin; l <= L; ++l) {
            Level &V = P.lv[l];
            fs.box0[l - lmin] = tot;
            fs.ff_ofs[l - lmin] = V.ff_ofs.as<int32_t>();
            fs.slot_base[l - lmin] = V.slot_base;
            fs.L[l - lmin] = V.L.p;
            tot += V.nbox;
        }
        fs.box0[L - lmin + 1] = tot;
        tm.begin(ST_SUMS, s, ev);
        k_sum_far_all<T><<<(unsigned)tot, TPB, 0, s>>>(fs, yb, blk, ncol * P2);
        FMB_LAUNCH_CHECK();
        tm.end(ST_SUMS, s, ev);
        return true;
    }
    for (int l = 3; l <= L; ++l) {
        Level &V = P.lv[l];
        if (step != k++) continue;
        if (l <= lmin) return true;
        if (P.hf) {
            tm.begin(ST_L2L, s, ev);
            hf_l2l<T>(P, l, nrhs, s);
            tm.end(ST_L2L, s, ev);
            return true;
        }
        if (V.ntiles_l2l == 0) return true;
        Level &U = P.lv[l - 1];
        tm.begin(ST_L2L, s, ev);
        for (int r0 = 0; r0 < nrhs; r0 += cw)
            launch_translate<T>(V.tiles_l2l.as<Tile>(), V.ntiles_l2l, V.by_octant.as<int32_t>(), V.parent.as<int32_t>(),
                                V.l2l.as<T>(), (const T *)U.L.p + roff(r0), (T *)V.L.p + roff(r0), KR,
                                3 * std::min(cw, nrhs - r0), blkR, os, s, 2, 1, bf3 ? V.l2l_hi.p : nullptr,
                                V.l2l_lo.p);
        tm.end(ST_L2L, s, ev, (nrhs + cw - 1) / cw);
        return true;
    }
    // Step 4: local expansions at the targets, then the near sum
    if (step == k++) {
        if (!far) {
            // local-only plan: the near sum accumulates onto zero
            k_zero<T><<<gridn((int64_t)nrhs * n * 3), TPB, 0, s>>>(ys, (int64_t)nrhs * n * 3);
            FMB_LAUNCH_CHECK();
            return true;
        }
        // chunk of right-hand sides per block while their local expansions fit ~24 KB of LDS
        const size_t lrhs = (size_t)3 * P2 * sizeof(cx<T>);
        const int rc = (nrhs >= 8 && 8 * lrhs <= 24576) ? 8 : ((nrhs >= 4 && 4 * lrhs <= 24576) ? 4 : 1);
        const size_t sh = (size_t)rc * lrhs + (size_t)64 * p * sizeof(cx<T>);
        const dim3 grid((unsigned)LL.nbox, (unsigned)((nrhs + rc - 1) / rc));
        auto kern = rc == 8 ? k_l2p<T, 8> : (rc == 4 ? k_l2p<T, 4> : k_l2p<T, 1>);
        tm.begin(ST_L2P, s, ev);
        kern<<<grid, 64, sh, s>>>(LL.start.as<int32_t>(), LL.center.as<double>(), P.spts.as<double>(), n, p, P.k_re,
                                  P.k_im, P.inv_alpha.as<double>() + (size_t)L * p, P.btab.as<T>(), nrhs, P.nrhs_max,
                                  LL.L.as<cx<T>>(), ys);
        FMB_LAUNCH_CHECK();
        tm.end(ST_L2P, s, ev);
        return true;
    }
    if (step == k++) {
        if (P.fuse_p2p) return true;           // the two-product runner launches both near fields at once
        tm.begin(ST_P2P, s, ev);
        if (sizeof(T) == sizeof(float)) {
            const bool lossy = P.k_im != 0.0;
            const int rc = nrhs >= 8 ? 8 : (nrhs >= 4 ? 4 : (nrhs >= 2 ? 2 : 1));
            decltype(&k_p2p32<true, 1>) kern;
            switch (rc) {
                case 8: kern = lossy ? k_p2p32<true, 8> : k_p2p32<false, 8>; break;
                case 4: kern = lossy ? k_p2p32<true, 4> : k_p2p32<false, 4>; break;
                case 2: kern = lossy ? k_p2p32<true, 2> : k_p2p32<false, 2>; break;
                default: kern = lossy ? k_p2p32<true, 1> : k_p2p32<false, 1>; break;
            }
            if (!far) {
                switch (rc) {
                    case 8: kern = k_p2p32_cut<8>; break;
                    case 4: kern = k_p2p32_cut<4>; break;
                    case 2: kern = k_p2p32_cut<2>; break;
                    default: kern = k_p2p32_cut<1>; break;
                }
            }
            kern<<<dim3((unsigned)LL.nbox, (unsigned)((nrhs + rc - 1) / rc)), TPB, 0, s>>>(
                (int)LL.nbox, nrhs, LL.start.as<int32_t>(), LL.nbr.as<int32_t>(), LL.center.as<double>(),
                P.spts.as<double>(), P.snrm.as<double>(), P.stri.as<int32_t>(), (const cx<float> *)src, n, P.k_re,
                P.k_im, (float)std::min(P.rcut2, 1e30), (cx<float> *)ys);
        } else {
            k_p2p<T><<<dim3((unsigned)LL.nbox, nrhs), TPB, 0, s>>>(
                LL.start.as<int32_t>(), LL.nbr.as<int32_t>(), P.spts.as<double>(), P.snrm.as<double>(),
                P.stri.as<int32_t>(), src, n, P.k_re, P.k_im, P.rcut2, ys);
        }
        FMB_LAUNCH_CHECK();
        tm.end(ST_P2P, s, ev);
        return true;
    }
    if (step != k++) return false;
    if (P.corr_mode != FMB_CORR_NONE) {
        // back to user order with the self-triangle terms added in the same pass
        tm.begin(ST_CORR, s, ev);
        scatter_with_corrections(P, ys, a, b, y, nrhs, s);
        tm.end(ST_CORR, s, ev);
    } else {
        tm.begin(ST_SCATTER, s, ev);
        k_scatter_out<T><<<gridn(n), TPB, 0, s>>>(ys, P.perm.as<int32_t>(), n, nrhs, y);
        FMB_LAUNCH_CHECK();
        tm.end(ST_SCATTER, s, ev);
    }
    return true;
}

}  // namespace

// target job count per launch: about 12 resident blocks on each of the 256 CUs
constexpr int64_t EP_BLOCKS = 3072;

void build_tiles(Plan &P, hipStream_t s) {
    const int L = P.depth;
    auto upload = [&](std::vector<Tile> &v, DevBuf &buf, int64_t &cnt) {
        cnt = (int64_t)v.size();
        buf.alloc(std::max<size_t>(1, v.size()) * sizeof(Tile));
        if (!v.empty())
            FMB_CHECK_HIP(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(Tile), hipMemcpyHostToDevice, s));
    };
    // entries per tile.  Operator-stationary jobs hold up to OS_MAXCOLS columns;
    // shorter jobs are used until a level spreads over about EP_BLOCKS blocks:
    // a job walks its columns one 16-column chunk after another, so the level's
    // time is set by the longest chain of gathered loads, not by operator traffic.
    const bool os = use_os(P.precision, P.order, P.nrhs_max);
    const int cols = use_bf3(P) ? bf3_job_cols(P.order)
                                : (os ? OS_MAXCOLS
                                      : (use_big(P.precision, 2 * P.P2)
                                             ? (P.precision == FMB_FP64 ? big_n<double>() : big_n<float>())
                                             : TN));
    const int cw = translate_rhs_chunk(P);
    const int ep_max = std::max(1, cols / (3 * cw));
    const int ep_min = os ? std::max(1, OS_COLS / (3 * cw)) : ep_max;
    auto ep_for = [&](int64_t total) {
        int64_t e = total / EP_BLOCKS;
        return (int)std::max<int64_t>(ep_min, std::min<int64_t>(ep_max, e));
    };
    auto chunk = [](std::vector<Tile> &v, int ep, int op, int first, int count) {
        for (int q = 0; q < count; q += ep) v.push_back(Tile{op, first + q, std::min(ep, count - q)});
    };
    for (int l = std::max(2, P.far_lmin); l <= L; ++l) {
        Level &V = P.lv[l];
        std::vector<Tile> t;
        const int e2l = ep_for(V.nff);
        for (int o = 0; o < N_M2L_OPS; ++o) chunk(t, e2l, o, V.op_start[o], V.op_start[o + 1] - V.op_start[o]);
        upload(t, V.tiles_m2l, V.ntiles_m2l);
        if (l < L) {
            Level &C = P.lv[l + 1];
            std::vector<Tile> u;
            const int e = ep_for(C.nbox);
            for (int o = 0; o < 8; ++o) chunk(u, e, o, C.oct_start[o], C.oct_start[o + 1] - C.oct_start[o]);
            upload(u, V.tiles_m2m, V.ntiles_m2m);
        }
        if (l >= 3 && l > P.far_lmin) {
            std::vector<Tile> u;
            const int e = ep_for(V.nbox);
            for (int o = 0; o < 8; ++o) chunk(u, e, o, V.oct_start[o], V.oct_start[o + 1] - V.oct_start[o]);
            upload(u, V.tiles_l2l, V.ntiles_l2l);
        }
    }
    FMB_CHECK_HIP(hipStreamSynchronize(s));
}

void split_operators(Plan &P, hipStream_t s) {
    if (!use_bf3(P)) return;
    const int KR = 2 * P.P2, RT = (KR + 15) / 16, KS = (KR + 31) / 32;
    auto split = [&](const DevBuf &T, int nops, DevBuf &hi, DevBuf &lo) {
        if (!T.p) return;
        const int64_t total = (int64_t)nops * RT * KS * 64;
        hi.alloc(total * sizeof(bf16x8));
        lo.alloc(total * sizeof(bf16x8));
        k_split_bf16<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(T.as<float>(), nops, KR, RT, KS, hi.as<bf16x8>(),
                                                                      lo.as<bf16x8>());
        FMB_LAUNCH_CHECK();
    };
    for (int l = std::max(2, P.far_lmin); l <= P.depth; ++l) {
        Level &V = P.lv[l];
        split(V.m2l, N_M2L_OPS, V.m2l_hi, V.m2l_lo);
        if (l < P.depth) split(V.m2m, 8, V.m2m_hi, V.m2m_lo);
        if (l >= 3 && l > P.far_lmin) split(V.l2l, 8, V.l2l_hi, V.l2l_lo);
    }
    FMB_CHECK_HIP(hipStreamSynchronize(s));
}

void alloc_workspace(Plan &P) {
    const size_t esz = P.precision == FMB_FP64 ? sizeof(cx<double>) : sizeof(cx<float>);
    const int64_t blk = (int64_t)P.nrhs_max * 3 * P.P2;
    if (P.hf) {
        // order per level; the translations need no slot buffer
        for (int l = std::max(2, P.far_lmin); l <= P.depth; ++l) {
            Level &V = P.lv[l];
            const int64_t b = (int64_t)P.nrhs_max * 3 * V.p * V.p;
            V.M.alloc((size_t)V.nbox * b * esz);
            V.L.alloc((size_t)V.nbox * b * esz);
        }
        P.ybuf.alloc(256);
        P.src.alloc((size_t)P.nrhs_max * P.n * 7 * esz);
        P.ys.alloc((size_t)P.nrhs_max * P.n * 3 * esz);
        return;
    }
    // S|R slots of all levels side by side (they are written in one run of
    // launches); the S|S slots of the upward pass reuse the front of the buffer
    int64_t slots = 1, sr = 0;
    for (int l = std::max(2, P.far_lmin); l <= P.depth; ++l) {
        Level &V = P.lv[l];
        V.M.alloc((size_t)V.nbox * blk * esz);
        V.L.alloc((size_t)V.nbox * blk * esz);
        V.slot_base = sr;
        sr += V.nff;
        if (l < P.depth) slots = std::max<int64_t>(slots, P.lv[l + 1].nbox);
    }
    slots = std::max(slots, sr);
    P.ybuf.alloc((size_t)slots * blk * esz);
    P.src.alloc((size_t)P.nrhs_max * P.n * 7 * esz);
    P.ys.alloc((size_t)P.nrhs_max * P.n * 3 * esz);
}

hipEvent_t StageTimer::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e;
    FMB_CHECK_HIP(hipEventCreate(&e));
    return e;
}

void StageTimer::begin(int st, hipStream_t s, hipEvent_t &e0) {
    if (!(mask >> st & 1u)) return;
    e0 = get();
    FMB_CHECK_HIP(hipEventRecord(e0, s));
}

void StageTimer::end(int st, hipStream_t s, hipEvent_t e0, int nk) {
    if (!(mask >> st & 1u)) return;
    hipEvent_t e1 = get();
    FMB_CHECK_HIP(hipEventRecord(e1, s));
    pending[st].push_back({e0, e1});
    pending_nk[st].push_back(nk);
    if (pending[st].size() > 4096) collect();
}

void StageTimer::collect() {
    for (int st = 0; st < ST_COUNT; ++st) {
        for (size_t i = 0; i < pending[st].size(); ++i) {
            auto &pr = pending[st][i];
            FMB_CHECK_HIP(hipEventSynchronize(pr.second));
            float ms_ = 0.f;
            FMB_CHECK_HIP(hipEventElapsedTime(&ms_, pr.first, pr.second));
            ms[st] += ms_;
            launches[st] += pending_nk[st][i];
            pool.push_back(pr.first);
            pool.push_back(pr.second);
        }
        pending[st].clear();
        pending_nk[st].clear();
    }
}

void StageTimer::reset() {
    collect();
    for (int st = 0; st < ST_COUNT; ++st) {
        ms[st] = 0;
        launches[st] = 0;
    }
}

StageTimer::~StageTimer() {
    for (int st = 0; st < ST_COUNT; ++st)
        for (auto &pr : pending[st]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

// The adjoint product shares the forward steps from P2M through the last
// R|R level (its sources are monopole charges in the forward record layout);
// gather, L2P, P2P and the return to user order are its own.
static bool adjoint_step(Plan &P, const void *y, void *abar, void *bbar, int nrhs, hipStream_t s, int step) {
    const int nmid = 3 + 2 * std::max(P.depth - 2, 0);
    StageTimer &tm = P.timer;
    hipEvent_t ev = nullptr;
    if (step == 0) {
        tm.begin(ST_GATHER, s, ev);
        adjoint_gather(P, y, nrhs, s);
        tm.end(ST_GATHER, s, ev);
        return true;
    }
    if (step <= nmid) {
        if (P.precision == FMB_FP64) return matvec_step<double>(P, nullptr, nullptr, nullptr, nrhs, s, step);
        return matvec_step<float>(P, nullptr, nullptr, nullptr, nrhs, s, step);
    }
    if (step == nmid + 1) {
        tm.begin(ST_L2P, s, ev);
        adjoint_l2p(P, nrhs, s);
        tm.end(ST_L2P, s, ev);
        return true;
    }
    if (step == nmid + 2) {
        tm.begin(ST_P2P, s, ev);
        adjoint_p2p(P, nrhs, s);
        tm.end(ST_P2P, s, ev);
        return true;
    }
    if (step == nmid + 3) {
        tm.begin(ST_CORR, s, ev);
        adjoint_finish(P, y, abar, bbar, nrhs, s);
        tm.end(ST_CORR, s, ev);
        return true;
    }
    return false;
}

static bool run_step(Plan &P, const void *a, const void *b, void *y, int nrhs, hipStream_t s, int step) {
    if (P.precision == FMB_FP64)
        return matvec_step<double>(P, (const cx<double> *)a, (const cx<double> *)b, (cx<double> *)y, nrhs, s, step);
    return matvec_step<float>(P, (const cx<float> *)a, (const cx<float> *)b, (cx<float> *)y, nrhs, s, step);
}

void run_matvec(Plan &P, const void *a, const void *b, void *y, int nrhs, hipStream_t s) {
    for (int st = 0; run_step(P, a, b, y, nrhs, s, st); ++st) {
    }
}

void run_matvec_adjoint(Plan &P, const void *y, void *abar, void *bbar, int nrhs, hipStream_t s) {
    adjoint_prepare(P);
    for (int st = 0; adjoint_step(P, y, abar, bbar, nrhs, s, st); ++st) {
    }
}

// the two plans of one BEM application share their nodes and octree when both are
// FP32 over the same points at the same depth.  When the interior plan is local only
// (its product is a cut near field and little else), both near fields run as one
// launch.  When both plans have far fields, their products overlap on two streams,
// and joining them around one near-field launch measured slower (the 60k-node torus:
// 316 against 303 ms per mixed solve), so they stay apart.
static bool p2p_fusable(const Plan &P0, const Plan &P1) {
    return P0.precision == FMB_FP32 && P1.precision == FMB_FP32 && &P0 != &P1 && P0.n == P1.n &&
           P0.depth == P1.depth && P0.lv[P0.depth].nbox == P1.lv[P1.depth].nbox && P0.k_im == 0.0 &&
           P1.k_im > 0.0 && P0.far_on() && !P1.far_on() && P0.lo[0] == P1.lo[0] && P0.lo[1] == P1.lo[1] &&
           P0.lo[2] == P1.lo[2] && P0.ext == P1.ext;
}

// two events per device and host thread for the join around the fused near field
static hipEvent_t *pair_events() {
    static thread_local std::map<int, std::array<hipEvent_t, 2>> evs;
    int dev = 0;
    FMB_CHECK_HIP(hipGetDevice(&dev));
    auto it = evs.find(dev);
    if (it == evs.end()) {
        std::array<hipEvent_t, 2> e{};
        for (auto &x : e) FMB_CHECK_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming));
        it = evs.emplace(dev, e).first;
    }
    return it->second.data();
}

static void launch_p2p_pair(Plan &P0, Plan &P1, int nrhs, hipStream_t s) {
    Level &LL = P0.lv[P0.depth];
    hipEvent_t ev = nullptr;
    P0.timer.begin(ST_P2P, s, ev);
    k_p2p32_pair<<<dim3((unsigned)LL.nbox, (unsigned)nrhs), TPB, 0, s>>>(
        (int)LL.nbox, nrhs, LL.start.as<int32_t>(), LL.nbr.as<int32_t>(), LL.center.as<double>(),
        P0.spts.as<double>(), P0.snrm.as<double>(), P0.stri.as<int32_t>(), P0.src.as<cx<float>>(),
        P1.src.as<cx<float>>(), P0.n, P0.k_re, P1.k_re, P1.k_im, (float)std::min(P1.rcut2, 1e30),
        P0.ys.as<cx<float>>(), P1.ys.as<cx<float>>());
    FMB_LAUNCH_CHECK();
    P0.timer.end(ST_P2P, s, ev);
}

void run_matvec_pair(Plan &P0, const void *a0, const void *b0, void *y0, hipStream_t s0, Plan &P1, const void *a1,
                     const void *b1, void *y1, hipStream_t s1, int nrhs) {
    // the near-field step (the same index in both plans: gather, P2M, the S|S levels, S|R, its sums,
    // the R|R levels, L2P, then P2P)
    const bool fuse = p2p_fusable(P0, P1);
    const int p2p_step = 2 * P0.depth + 1;
    P0.fuse_p2p = P1.fuse_p2p = fuse;
    struct Reset {
        Plan &a, &b;
        ~Reset() { a.fuse_p2p = b.fuse_p2p = false; }
    } reset{P0, P1};
    bool more0 = true, more1 = true;
    for (int st = 0; more0 || more1; ++st) {
        if (more0) more0 = run_step(P0, a0, b0, y0, nrhs, s0, st);
        if (more1) more1 = run_step(P1, a1, b1, y1, nrhs, s1, st);
        if (fuse && st == p2p_step) {
            // s0 waits for s1's L2P, runs both near fields, and s1 waits for that
            hipEvent_t *ev = pair_events();
            if (s0 != s1) {
                FMB_CHECK_HIP(hipEventRecord(ev[0], s1));
                FMB_CHECK_HIP(hipStreamWaitEvent(s0, ev[0], 0));
            }
            launch_p2p_pair(P0, P1, nrhs, s0);
            if (s0 != s1) {
                FMB_CHECK_HIP(hipEventRecord(ev[1], s0));
                FMB_CHECK_HIP(hipStreamWaitEvent(s1, ev[1], 0));
            }
        }
    }
}

}  // namespace fmb
