// The adjoint product (a_bar, b_bar) = Op_k^H y of one plan.
//
// Op_k(a, b)_alpha = sum_beta w_beta [ K(n_beta; s_beta, s_alpha) . a_beta + g b_beta ] (eq. 2.12 with the
// point rule of eq. 2.8) is bilinear in (y, (a, b)); its transpose, written per
// source node beta with d = s_beta - s_alpha and f = (ikR - 1) e^{ikR} / (4 pi R^3),
//   a_bar_beta = w_beta sum_alpha f [ d (n_beta . y_alpha) - (n_beta . d) y_alpha - n_beta (d . y_alpha) ]
//   b_bar_beta = w_beta sum_alpha g y_alpha,
// needs, at every node, the potentials F_c(s) = sum_alpha g(s, s_alpha) y_alpha,c of
// plain monopole charges and their gradients H_ic = d_i F_c:
//   a_bar = w (H n - H^T n - n tr H),   b_bar = w F.
// So the adjoint is the same fast multipole method with monopole sources (the
// forward P2M with charges in the b slot, and the same S|S, S|R and R|R passes),
// an L2P that also evaluates gradients, a near field that accumulates value and
// gradient, and the transposed self-triangle blocks.  The conjugate transpose is
// taken as conj(Op^T conj(y)).
#include "basis.h"
#include "plan.h"

namespace fmb {

namespace {

constexpr int GTPB = 256;
constexpr int ATPB = 256;       // near-field block: targets on lanes, source slices on spare lanes (256: 8% faster than 128 in FP32)

inline unsigned grid_for(int64_t m, int tpb) { return (unsigned)((m + tpb - 1) / tpb); }

// Source records in the forward layout (w a, w b, w n.a) carrying conj(y) as
// the monopole charges: (0, conj(y), 0), Morton order.
template <typename T>
__global__ void k_adj_gather(const cx<T> *__restrict__ y, const int32_t *__restrict__ perm, int64_t n, int nrhs,
                             cx<T> *__restrict__ src) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t u = perm[i];
    for (int r = 0; r < nrhs; ++r) {
        const cx<T> *Y = y + ((int64_t)r * n + u) * 3;
        cx<T> *o = src + ((int64_t)r * n + i) * 7;
        const cx<T> z = mk(T(0), T(0));
        o[0] = z;
        o[1] = z;
        o[2] = z;
        o[3] = conj(Y[0]);
        o[4] = conj(Y[1]);
        o[5] = conj(Y[2]);
        o[6] = z;
    }
}

// Far field at the nodes of one leaf (blockIdx.x) for one right-hand side
// (blockIdx.y): F_c = sum_nm L_nm,c R_n^m(s - X) and grad F_c.  The gradient
// of a local expansion of degree < p is one of degree <= p: the plan's
// gradient table gives grad R_n^{mu} as k times two terms per component
// (d_z, d_+ = d_x + i d_y, d_- = d_x - i d_y, each from R_{n+-1}) for mu = -m
// at coefficient (n, m), so grad R_n^m is read from the row of (n, -m).  Per
// channel the block scatters L into the three coefficient sets D_x, D_y, D_z
// (one thread per set, fixed order), then every thread evaluates L and the
// three sets at its nodes with one pass of the Legendre recurrence.
// out[(r n + i) 12 + e]: e = c for F_c, e = 3 + 3 i + c for d_i F_c.
template <typename T>
__global__ void __launch_bounds__(64) k_adj_l2p(const int32_t *__restrict__ start, const double *__restrict__ center,
                                                const double *__restrict__ spts, int64_t n, int p, double k_re,
                                                double k_im, const double *__restrict__ inv_alpha,
                                                const T *__restrict__ tab, const int32_t *__restrict__ gix,
                                                const int32_t *__restrict__ gath, int nrhs_max,
                                                const cx<T> *__restrict__ Lc, cx<T> *__restrict__ out) {
    extern __shared__ unsigned char smem[];
    const int P2 = p * p, N = p, NN = (N + 1) * (N + 1), NS = NN + 1;
    const BasisTab<T> bt = basis_tab(tab, gix, N, P2);
    cx<T> *D = reinterpret_cast<cx<T> *>(smem);        // [4][NS]: L, D_x, D_y, D_z of one channel
    cx<T> *jb = D + 4 * NS;                             // [blockDim][N + 1]
    const int box = blockIdx.x, r = blockIdx.y;
    const int s0 = start[box], s1 = start[box + 1];
    const cx<T> k = mk((T)k_re, (T)k_im);
    const double X[3] = {center[3 * box], center[3 * box + 1], center[3 * box + 2]};
    const cx<T> *Lb = Lc + ((int64_t)box * nrhs_max + r) * 3 * P2;
    const int32_t *gptr = gath, *gent = gath + NN + 1;
    for (int c = 0; c < 3; ++c) {
        __syncthreads();                                // the previous channel's evaluation is done
        for (int t = threadIdx.x; t < NS; t += blockDim.x) {
            cx<T> v = mk(T(0), T(0));
            if (t < P2) {
                int nn = 0;
                while ((nn + 1) * (nn + 1) <= t) ++nn;
                v = (T)inv_alpha[nn] * Lb[c * P2 + t];
            }
            D[t] = v;
        }
        __syncthreads();
        // D_x, D_y, D_z: every R-table entry o gathers the gradient terms that land on it, in increasing
        // source index (the terms of coefficient idx: slots 0-1 d_z, 2-3 d_+, 4-5 d_- of its gradient row)
        for (int o = threadIdx.x; o < NS; o += blockDim.x) {
            cx<T> ax = mk(T(0), T(0)), ay = mk(T(0), T(0)), az = mk(T(0), T(0));
            if (o < NN)
                for (int e = gptr[o]; e < gptr[o + 1]; ++e) {
                    const int pk = gent[e];
                    const int idx = pk & 2047, row = (pk >> 11) & 2047, slot = pk >> 22;
                    const T co = bt.gco[(int64_t)row * 6 + slot];
                    const cx<T> l = k * D[idx];
                    if (slot < 2) {
                        az += co * l;                   // d_z
                    } else {
                        ax += co * (T(0.5) * l);        // d_x = (d_+ + d_-) / 2
                        const cx<T> h = mk(T(0.5) * l.im, T(-0.5) * l.re);
                        if (slot < 4) ay += co * h;     // d_y = (d_+ - d_-) / 2i
                        else ay -= co * h;
                    }
                }
            D[NS + o] = ax;
            D[2 * NS + o] = ay;
            D[3 * NS + o] = az;
        }
        __syncthreads();
        for (int i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
            double d[3];
            for (int q = 0; q < 3; ++q) d[q] = spts[3 * (int64_t)i + q] - X[q];
            const double rr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double ir = rr > 0 ? 1.0 / rr : 0.0;
            cx<T> *J = jb + threadIdx.x * (N + 1);
            sph_bessel_j(mk((T)(k_re * rr), (T)(k_im * rr)), N, J);
            const T x = rr > 0 ? (T)(d[2] * ir) : T(1);
            const cx<T> w = mk((T)(d[0] * ir), (T)(d[1] * ir));
            cx<T> acc[4] = {mk(T(0), T(0)), mk(T(0), T(0)), mk(T(0), T(0)), mk(T(0), T(0))};
            cx<T> wm = mk(T(1), T(0));
            for (int m = 0; m <= N; ++m) {
                if (m > 0) wm = wm * w;
                const T qmm = bt.qmm[m];
                const T sgn = (m & 1) ? T(-1) : T(1);
                T q2 = 0, q1 = qmm;
                for (int nn = m; nn <= N; ++nn) {
                    T qv;
                    if (nn == m) qv = qmm;
                    else if (nn == m + 1) qv = bt.q1[m] * x * qmm;
                    else qv = bt.la[nn * (N + 1) + m] * (x * q1 - bt.lb[nn * (N + 1) + m] * q2);
                    if (nn > m) {
                        q2 = q1;
                        q1 = qv;
                    }
                    const cx<T> Y = (sgn * qv) * wm;
                    const cx<T> Rp = J[nn] * Y;
                    const int ip = nn * nn + nn + m;
#pragma unroll
                    for (int s = 0; s < 4; ++s) acc[s] += D[s * NS + ip] * Rp;
                    if (m > 0) {
                        const cx<T> Rm = J[nn] * conj(Y);
                        const int im = nn * nn + nn - m;
#pragma unroll
                        for (int s = 0; s < 4; ++s) acc[s] += D[s * NS + im] * Rm;
                    }
                }
            }
            cx<T> *o = out + ((int64_t)r * n + i) * 12;
            o[c] = acc[0];
            for (int q = 0; q < 3; ++q) o[3 + 3 * q + c] = acc[1 + q];
        }
    }
}

// Near field of the adjoint: for each node beta of the leaf and every node
// alpha of the leaf and its neighbours outside beta's triangle, with
// d = s_beta - s_alpha, add g q_alpha,c to F_c and f d_i q_alpha,c to d_i F_c
// (q = conj(y) from the source records).  Targets on lanes; spare lanes take
// slices of the sources, summed in LDS at the end in a fixed order.
template <typename T>
struct AdjTile {
    T pos[ATPB][3];                 // relative to the target leaf's centre
    int32_t tri[ATPB];
    cx<T> q[ATPB][3];
};

template <typename T>
__global__ void __launch_bounds__(ATPB) k_adj_p2p(const int32_t *__restrict__ start, const int32_t *__restrict__ nbr,
                                                  const double *__restrict__ center,
                                                  const double *__restrict__ spts, const int32_t *__restrict__ stri,
                                                  const cx<T> *__restrict__ src, int64_t n, double k_re, double k_im,
                                                  double rcut2, cx<T> *__restrict__ out) {
    __shared__ AdjTile<T> tile;
    __shared__ int32_t nb_start[28], nb_box[27];
    __shared__ int n_nb;
    __shared__ cx<T> red[ATPB][12];
    const int box = blockIdx.x, r = blockIdx.y;
    const int t0 = start[box], t1 = start[box + 1];
    const int nt = t1 - t0;
    if (threadIdx.x == 0) {
        int c = 0, tot = 0;
        for (int s = 0; s < 27; ++s) {
            const int q = nbr[box * 27 + s];
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
    // coordinates relative to this leaf's centre: the differences of near pairs in T keep full precision
    const double C[3] = {center[3 * box], center[3 * box + 1], center[3 * box + 2]};
    const T kr = (T)k_re, ki = (T)k_im;
    const T inv4pi = T(0.07957747154594766788);
    for (int tc0 = 0; tc0 < nt; tc0 += ATPB) {
        const int ntc = min(ATPB, nt - tc0);
        const int S = ATPB / ntc;
        const int ti = threadIdx.x % ntc, sl = threadIdx.x / ntc;
        const bool active = sl < S;
        const int64_t ig = t0 + tc0 + ti;
        T tp[3] = {0, 0, 0};
        int32_t ttri = -1;
        if (active) {
            for (int q = 0; q < 3; ++q) tp[q] = (T)(spts[3 * ig + q] - C[q]);
            ttri = stri[ig];
        }
        cx<T> acc[12];
        for (int e = 0; e < 12; ++e) acc[e] = mk(T(0), T(0));
        for (int base = 0; base < ns_total; base += ATPB) {
            const int cnt = min(ATPB, ns_total - base);
            __syncthreads();
            for (int j = threadIdx.x; j < cnt; j += blockDim.x) {
                const int u = base + j;
                int b = 0;
                while (nb_start[b + 1] <= u) ++b;
                const int64_t sidx = start[nb_box[b]] + (u - nb_start[b]);
                for (int q = 0; q < 3; ++q) tile.pos[j][q] = (T)(spts[3 * sidx + q] - C[q]);
                tile.tri[j] = stri[sidx];
                const cx<T> *sr = src + ((int64_t)r * n + sidx) * 7;
                for (int q = 0; q < 3; ++q) tile.q[j][q] = sr[3 + q];
            }
            __syncthreads();
            if (!active) continue;
            for (int j = sl; j < cnt; j += S) {
                if (tile.tri[j] == ttri) continue;
                const T dx = tp[0] - tile.pos[j][0], dy = tp[1] - tile.pos[j][1], dz = tp[2] - tile.pos[j][2];
                const T R2 = dx * dx + dy * dy + dz * dz;
                if (R2 > rcut2) continue;       // damped below the cutoff (local-only lossy plans)
                const T iR = fast_rsqrt(R2);
                const T R = R2 * iR;
                T sn, cs;
                fast_sincos(kr * R, &sn, &cs);
                const T ex = ki != T(0) ? fast_exp(-ki * R) : T(1);
                const cx<T> g = (inv4pi * iR) * mk(ex * cs, ex * sn);
                const cx<T> f = (iR * iR) * (mk(-ki * R - T(1), kr * R) * g);
                const cx<T> fd[3] = {dx * f, dy * f, dz * f};
                for (int c = 0; c < 3; ++c) {
                    const cx<T> q = tile.q[j][c];
                    acc[c] += g * q;
                    for (int i = 0; i < 3; ++i) acc[3 + 3 * i + c] += fd[i] * q;
                }
            }
        }
        __syncthreads();
        for (int e = 0; e < 12; ++e) red[threadIdx.x][e] = acc[e];
        __syncthreads();
        if ((int)threadIdx.x < ntc) {
            cx<T> *o = out + ((int64_t)r * n + t0 + tc0 + threadIdx.x) * 12;
            for (int e = 0; e < 12; ++e) {
                cx<T> s = mk(T(0), T(0));
                for (int q = 0; q < S; ++q) s += red[q * ntc + threadIdx.x][e];
                o[e] += s;
            }
        }
    }
}

// Back to user order: a_bar = conj(w (H n - H^T n - n tr H) + corrections),
// b_bar = conj(w F + corrections), where the transposed self-triangle blocks of
// node beta (triangle t, beta the j-th node of t) add, for every node alpha of t,
//   dV (n_beta . q_alpha) - (n_beta . dV) q_alpha - n_beta (dV . q_alpha)  to a_bar,
//   dG q_alpha  to b_bar,  with dV = dV[alpha][j], dG = dG[alpha][j], q = conj(y).
template <typename T>
__global__ void k_adj_finish(const cx<T> *__restrict__ fh, const int32_t *__restrict__ iperm,
                             const double *__restrict__ sw, const double *__restrict__ unrm,
                             const cx<T> *__restrict__ y, const int32_t *__restrict__ point_tri,
                             const int32_t *__restrict__ tri_nodes, const cx<double> *__restrict__ cv,
                             const cx<double> *__restrict__ cg, int64_t n, int m, int nrhs, cx<T> *__restrict__ abar,
                             cx<T> *__restrict__ bbar) {
    const int64_t be = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (be >= n) return;
    const int64_t im = iperm[be];
    const double w = sw[im];
    const double nb[3] = {unrm[3 * be], unrm[3 * be + 1], unrm[3 * be + 2]};
    int jb = -1;
    int32_t t = 0;
    if (tri_nodes) {
        t = point_tri[be];
        for (int j = 0; j < m; ++j)
            if (tri_nodes[(int64_t)t * m + j] == (int32_t)be) jb = j;
    }
    for (int r = 0; r < nrhs; ++r) {
        const int64_t off = (int64_t)r * n;
        const cx<T> *v = fh + (off + im) * 12;
        cx<double> F[3], H[3][3];
        for (int c = 0; c < 3; ++c) F[c] = mk((double)v[c].re, (double)v[c].im);
        for (int i = 0; i < 3; ++i)
            for (int c = 0; c < 3; ++c) H[i][c] = mk((double)v[3 + 3 * i + c].re, (double)v[3 + 3 * i + c].im);
        const cx<double> tr = H[0][0] + H[1][1] + H[2][2];
        cx<double> A[3], B[3];
        for (int i = 0; i < 3; ++i) {
            cx<double> hn = mk(0.0, 0.0), htn = mk(0.0, 0.0);
            for (int c = 0; c < 3; ++c) {
                hn += nb[c] * H[i][c];
                htn += nb[c] * H[c][i];
            }
            A[i] = w * (hn - htn - nb[i] * tr);
            B[i] = w * F[i];
        }
        if (jb >= 0) {
            for (int j = 0; j < m; ++j) {
                const int64_t al = tri_nodes[(int64_t)t * m + j];
                cx<double> q[3], dV[3];
                for (int i = 0; i < 3; ++i) {
                    const cx<T> yv = y[(off + al) * 3 + i];
                    q[i] = mk((double)yv.re, -(double)yv.im);
                    dV[i] = cv[(al * m + jb) * 3 + i];
                }
                const cx<double> dG = cg[al * m + jb];
                const cx<double> nq = nb[0] * q[0] + nb[1] * q[1] + nb[2] * q[2];
                const cx<double> nV = nb[0] * dV[0] + nb[1] * dV[1] + nb[2] * dV[2];
                const cx<double> Vq = dV[0] * q[0] + dV[1] * q[1] + dV[2] * q[2];
                for (int i = 0; i < 3; ++i) {
                    A[i] += dV[i] * nq - nV * q[i] - nb[i] * Vq;
                    B[i] += dG * q[i];
                }
            }
        }
        for (int i = 0; i < 3; ++i) {
            abar[(off + be) * 3 + i] = mk((T)A[i].re, (T)(-A[i].im));
            bbar[(off + be) * 3 + i] = mk((T)B[i].re, (T)(-B[i].im));
        }
    }
}

template <typename T>
void gather_t(Plan &P, const void *y, int nrhs, hipStream_t s) {
    k_adj_gather<T><<<grid_for(P.n, GTPB), GTPB, 0, s>>>((const cx<T> *)y, P.perm.as<int32_t>(), P.n, nrhs,
                                                          P.src.as<cx<T>>());
    FMB_LAUNCH_CHECK();
}

size_t l2p_lds(const Plan &P, int threads) {
    const size_t cs = P.precision == FMB_FP64 ? sizeof(cx<double>) : sizeof(cx<float>);
    const int N = P.order, NS = (N + 1) * (N + 1) + 1;
    return (size_t)(4 * NS + threads * (N + 1)) * cs;
}

template <typename T>
__global__ void k_adj_zero(cx<T> *__restrict__ x, int64_t m) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) x[i] = mk(T(0), T(0));
}

template <typename T>
void l2p_t(Plan &P, int nrhs, hipStream_t s) {
    if (!P.far_on()) {
        // local-only plan: the near field accumulates onto zero
        const int64_t m = (int64_t)nrhs * P.n * 12;
        k_adj_zero<T><<<grid_for(m, GTPB), GTPB, 0, s>>>(P.aws.as<cx<T>>(), m);
        FMB_LAUNCH_CHECK();
        return;
    }
    const Level &LL = P.lv[P.depth];
    const int threads = 64;
    const size_t sh = l2p_lds(P, threads);
    k_adj_l2p<T><<<dim3((unsigned)LL.nbox, (unsigned)nrhs), threads, sh, s>>>(
        LL.start.as<int32_t>(), LL.center.as<double>(), P.spts.as<double>(), P.n, P.order, P.k_re, P.k_im,
        P.inv_alpha.as<double>() + (size_t)P.depth * P.order, P.btab.as<T>(), P.bgix.as<int32_t>(),
        P.agath.as<int32_t>(), P.nrhs_max, LL.L.as<cx<T>>(), P.aws.as<cx<T>>());
    FMB_LAUNCH_CHECK();
}

template <typename T>
void p2p_t(Plan &P, int nrhs, hipStream_t s) {
    const Level &LL = P.lv[P.depth];
    k_adj_p2p<T><<<dim3((unsigned)LL.nbox, (unsigned)nrhs), ATPB, 0, s>>>(
        LL.start.as<int32_t>(), LL.nbr.as<int32_t>(), LL.center.as<double>(), P.spts.as<double>(),
        P.stri.as<int32_t>(), P.src.as<cx<T>>(),
        P.n, P.k_re, P.k_im, (double)(T)std::min(P.rcut2, 1e30), P.aws.as<cx<T>>());
    FMB_LAUNCH_CHECK();
}

template <typename T>
void finish_t(Plan &P, const void *y, void *abar, void *bbar, int nrhs, hipStream_t s) {
    const bool corr = P.corr_mode != FMB_CORR_NONE;
    k_adj_finish<T><<<grid_for(P.n, GTPB), GTPB, 0, s>>>(
        P.aws.as<cx<T>>(), P.iperm.as<int32_t>(), P.sw.as<double>(), P.unrm.as<double>(), (const cx<T> *)y,
        P.point_tri.as<int32_t>(), corr ? P.tri_nodes.as<int32_t>() : nullptr,
        corr ? P.corr_v.as<cx<double>>() : nullptr, corr ? P.corr_g.as<cx<double>>() : nullptr, P.n, (int)P.tri_m,
        nrhs, (cx<T> *)abar, (cx<T> *)bbar);
    FMB_LAUNCH_CHECK();
}

}  // namespace

void adjoint_prepare(Plan &P) {
    FMB_REQUIRE(l2p_lds(P, 64) <= 65536, "the adjoint's far-field evaluation supports orders up to 23 in FP64");
    const size_t cs = P.precision == FMB_FP64 ? sizeof(cx<double>) : sizeof(cx<float>);
    const size_t need = (size_t)P.nrhs_max * P.n * 12 * cs;
    if (P.aws.bytes < need) P.aws.alloc(need);
    if (!P.agath.p) {
        // invert the gradient table: for every R-table entry o < (N+1)^2, the (source coefficient, its
        // gradient row, slot) triples whose term lands on o, in increasing source coefficient
        const int N = P.order, NN = (N + 1) * (N + 1), P2 = N * N;
        std::vector<int32_t> gix((size_t)7 * P2);
        FMB_CHECK_HIP(hipMemcpy(gix.data(), P.bgix.p, gix.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        std::vector<int32_t> ptr(NN + 1, 0), pos, ent;
        std::vector<std::pair<int32_t, int32_t>> raw;
        for (int idx = 0; idx < P2; ++idx) {
            int nn = 0;
            while ((nn + 1) * (nn + 1) <= idx) ++nn;
            const int m = idx - nn * nn - nn, row = nn * nn + nn - m;
            for (int slot = 0; slot < 6; ++slot) {
                const int o = gix[(size_t)7 * row + slot];
                if (o < 0 || o >= NN) continue;               // the zero entry (N+1)^2
                raw.push_back({o, idx | (row << 11) | (slot << 22)});
                ++ptr[o + 1];
            }
        }
        for (int o = 0; o < NN; ++o) ptr[o + 1] += ptr[o];
        pos.assign(ptr.begin(), ptr.end() - 1);
        ent.resize(raw.size());
        for (const auto &e : raw) ent[pos[e.first]++] = e.second;
        std::vector<int32_t> buf(ptr);
        buf.insert(buf.end(), ent.begin(), ent.end());
        P.agath.alloc(buf.size() * sizeof(int32_t));
        FMB_CHECK_HIP(hipMemcpy(P.agath.p, buf.data(), buf.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
}

void adjoint_gather(Plan &P, const void *y, int nrhs, hipStream_t s) {
    if (P.precision == FMB_FP64) gather_t<double>(P, y, nrhs, s);
    else gather_t<float>(P, y, nrhs, s);
}

void adjoint_l2p(Plan &P, int nrhs, hipStream_t s) {
    if (P.precision == FMB_FP64) l2p_t<double>(P, nrhs, s);
    else l2p_t<float>(P, nrhs, s);
}

void adjoint_p2p(Plan &P, int nrhs, hipStream_t s) {
    if (P.precision == FMB_FP64) p2p_t<double>(P, nrhs, s);
    else p2p_t<float>(P, nrhs, s);
}

void adjoint_finish(Plan &P, const void *y, void *abar, void *bbar, int nrhs, hipStream_t s) {
    if (P.precision == FMB_FP64) finish_t<double>(P, y, abar, bbar, nrhs, s);
    else finish_t<float>(P, y, abar, bbar, nrhs, s);
}

}  // namespace fmb
