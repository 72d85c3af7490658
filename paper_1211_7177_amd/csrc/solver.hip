// BEM system of one scatterer (eqs. 2.9-2.13), the block preconditioner
// M = A_self (Sec. 3.1, eq. 3.2) and right-preconditioned flexible GMRES
// (eq. 3.1), all device-resident.
//
// Rows of node alpha (unknowns Phi = E_0, Psi = n x curl E_0):
//   r[0:3] = 1/2 Phi + Op_{k0}(Phi, -Psi)
//   r[3:6] = 1/2 T Phi - Op_{k1}(T Phi, -gamma Psi),   T = I + (1 - eps)/eps n n.
// M_alpha keeps the coincident-node self blocks (dV, dG) of both plans:
//   M = [[1/2 I + K(dV0), -dG0 I], [1/2 T - K(dV1) T, gamma dG1 I]],
//   K(V) a = n (V . a) - (n . V) a - V (n . a).
//
// fGMRES keeps the preconditioned directions z_j = M^{-1} v_j, orthogonalises
// A z_j against the basis by classical Gram-Schmidt, and updates a
// QR factorisation of the Hessenberg matrix with complex Givens rotations
//   c = |a| / sqrt(|a|^2 + |b|^2),  s = (a / |a|) conj(b) / sqrt(|a|^2 + |b|^2)
// (a = h_jj, b = h_{j+1,j}); |g_{j+1}| estimates the residual.  Several
// right-hand sides iterate in lockstep, each with its own Hessenberg matrix.
//
// Mixed mode (iterative refinement): r = b - A64 x with the FP64 plans, an
// inner fGMRES solves A32 d = r with the FP32 plans and FP32 Krylov vectors
// (inner products accumulated in FP64), x += d, until |r| <= tol |b|.
//
// Gram-Schmidt: one classical pass, then a second one only for the rhs where
// the first removed more than half of |A z|^2 (the DGKS criterion).  The inner
// FP32 solves of the mixed mode take the one pass only unless asked: they stop
// at a loose tolerance (about 5e-3), the FP32 basis keeps orthogonality far
// below that over a restart cycle, and the FP64 residual of the refinement
// decides the accuracy of the answer.  The two
// FMM products of each application run concurrently on two streams.
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include <complex>

#include "plan.h"

struct fmb_problem_s {
    fmb_plan_t p0 = nullptr, p1 = nullptr, p032 = nullptr, p132 = nullptr;
    int64_t n = 0;
    fmb::cx<double> eps, mu, gamma;
    double k0_re = 0, k0_im = 0;
    int nrhs_max = 1;
    // impedance boundary condition problems (eq. 2.25): one plan, three unknowns
    // per node, Psi replaced by -c n x (n x Phi) with c = i k0 / Z
    bool ibc = false;
    int nu = 6;                // unknowns per node: 6 (Phi, Psi) or 3 (Phi, ibc)
    fmb::cx<double> cibc;
    // several scatterers: plan pj[j] (and pj32[j]) holds scatterer j's nodes at
    // k_j; reg/loc map every node to its scatterer and its position there; the
    // interior staging block of scatterer j starts at element off[j] (per-rhs
    // stride nj[j] * 3).  One scatterer: J = 1, pj[0] = p1, no maps.
    int J = 1;
    fmb_plan_t pj[8] = {}, pj32[8] = {};
    fmb::DevBuf reg, loc;
    int64_t off[8] = {}, nj[8] = {};
    fmb::cx<double> tcj[8] = {}, gamj[8] = {};
    fmb::DevBuf minv;          // c128[n][6][6] (c128[n][3][3] for ibc)
    fmb::DevBuf minv32;        // c64[n][6][6], FP32 copy for the inner solves (FP32 plans only)
    // the blocks M themselves (the inverse of minv) and their FP32 copy, built at
    // the first solve that asks for the inner-GMRES preconditioner (precond = 2),
    // and that preconditioner's Krylov workspaces (FP64, FP32)
    fmb::DevBuf mfwd, mfwd32;
    std::shared_ptr<void> pg64, pg32;
    fmb::DevBuf upts;          // f64[n][3] user order
    // matvec staging [nrhs][n][3] for the two plans (FP64) and their FP32 copies
    fmb::DevBuf a0, b0, a1, b1, y0, y1;
    fmb::DevBuf a0s, b0s, a1s, b1s, y0s, y1s;
    // second stream (default priority) for the k1 product, and the fork/join events
    hipStream_t s2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool serial = false;       // both products on one stream (set per solve)
    bool adjoint = false;      // solves and applications use A^H and M^{-H} (set per solve)
    // Optionally (off by default) the two FMM products of an application,
    // captured once per precision and rhs count as a HIP graph and replayed on
    // the problem's own stream s1 (the caller's stream may be the legacy
    // default stream, which cannot be captured); ev_in / ev_out order s1 after
    // and before the caller's stream.  Eager launches, issued alternately to
    // the two streams, measured faster: the graph's second branch started
    // well after its first.
    bool graphs = false;
    hipStream_t s1 = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    struct PairGraph {
        hipGraphExec_t exec = nullptr;
        int nrhs = 0;
        bool serial = false;
    } g64, g32;
    ~fmb_problem_s() {
        for (PairGraph *g : {&g64, &g32})
            if (g->exec) (void)hipGraphExecDestroy(g->exec);
        for (hipEvent_t e : {ev_fork, ev_join, ev_in, ev_out})
            if (e) (void)hipEventDestroy(e);
        if (s2) (void)hipStreamDestroy(s2);
        if (s1) (void)hipStreamDestroy(s1);
    }
};

namespace fmb {

namespace {

constexpr int TPB = 256;
inline unsigned gridn(int64_t m) { return (unsigned)((m + TPB - 1) / TPB); }

__device__ inline void tmul(const double nv[3], double c, const cx<double> in[3], cx<double> out[3]) {
    // out = T in = in + c n (n . in)
    cx<double> d = nv[0] * in[0] + nv[1] * in[1] + nv[2] * in[2];
    for (int i = 0; i < 3; ++i) out[i] = in[i] + (c * nv[i]) * d;
}

template <typename T>
__device__ inline cx<T> narrow(cx<double> z) { return mk((T)z.re, (T)z.im); }
template <typename T>
__device__ inline cx<double> widen(cx<T> z) { return mk((double)z.re, (double)z.im); }

// Several scatterers: node alpha belongs to scatterer reg[alpha] = j, whose plan
// holds it at position loc[alpha]; the host plan holds every node.  Scatterer
// j's interior densities occupy the block [nrhs][n_j][3] starting at element
// off[j] of the interior staging arrays (the blocks of all scatterers fill
// n * 3 * nrhs_max elements, as the one scatterer does).  reg = loc = nullptr
// is the one-scatterer case.
constexpr int MAXJ = 8;
struct Regions {
    const int32_t *reg;
    const int32_t *loc;
    int64_t off[MAXJ];
    int64_t nj[MAXJ];
    cx<double> tc[MAXJ], gamma[MAXJ];
};

// element index of (rhs, node) in the interior staging arrays; j receives the scatterer
__device__ inline int64_t interior_at(const Regions &R, int64_t i, int64_t n, int &j) {
    const int64_t node = i % n, r = i / n;
    j = R.reg ? R.reg[node] : 0;
    const int64_t l = R.loc ? R.loc[node] : node;
    return R.off[j] + (r * R.nj[j] + l) * 3;
}

Regions regions_of(const fmb_problem_s &pb) {
    Regions R{};
    R.reg = pb.J > 1 ? pb.reg.as<int32_t>() : nullptr;
    R.loc = pb.J > 1 ? pb.loc.as<int32_t>() : nullptr;
    for (int j = 0; j < pb.J; ++j) {
        R.off[j] = pb.off[j];
        R.nj[j] = pb.nj[j];
        R.tc[j] = pb.tcj[j];
        R.gamma[j] = pb.gamj[j];
    }
    return R;
}

template <typename T>
__global__ void k_bem_split(const cx<T> *__restrict__ x, const double *__restrict__ nrm, int64_t n, int nrhs,
                            const Regions R, cx<T> *__restrict__ a0, cx<T> *__restrict__ b0,
                            cx<T> *__restrict__ a1, cx<T> *__restrict__ b1) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const int64_t node = i % n;
    int j;
    const int64_t ii = interior_at(R, i, n, j);
    const cx<T> tc = narrow<T>(R.tc[j]), gamma = narrow<T>(R.gamma[j]);
    const T nv[3] = {(T)nrm[3 * node], (T)nrm[3 * node + 1], (T)nrm[3 * node + 2]};
    const cx<T> *xi = x + i * 6;
    cx<T> phi[3] = {xi[0], xi[1], xi[2]}, psi[3] = {xi[3], xi[4], xi[5]};
    cx<T> d = nv[0] * phi[0] + nv[1] * phi[1] + nv[2] * phi[2];
    for (int c = 0; c < 3; ++c) {
        a0[i * 3 + c] = phi[c];
        b0[i * 3 + c] = -psi[c];
        a1[ii + c] = phi[c] + (nv[c] * tc) * d;
        b1[ii + c] = -(gamma * psi[c]);
    }
}

template <typename T>
__global__ void k_bem_combine(const cx<T> *__restrict__ x, const double *__restrict__ nrm, int64_t n, int nrhs,
                              const Regions R, const cx<T> *__restrict__ y0, const cx<T> *__restrict__ y1,
                              cx<T> *__restrict__ r) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const int64_t node = i % n;
    int j;
    const int64_t ii = interior_at(R, i, n, j);
    const cx<T> tc = narrow<T>(R.tc[j]);
    const T nv[3] = {(T)nrm[3 * node], (T)nrm[3 * node + 1], (T)nrm[3 * node + 2]};
    const cx<T> *xi = x + i * 6;
    cx<T> d = nv[0] * xi[0] + nv[1] * xi[1] + nv[2] * xi[2];
    for (int c = 0; c < 3; ++c) {
        cx<T> tphi = xi[c] + (nv[c] * tc) * d;
        r[i * 6 + c] = T(0.5) * xi[c] + y0[i * 3 + c];
        r[i * 6 + 3 + c] = T(0.5) * tphi - y1[ii + c];
    }
}

__global__ void k_to32(const cx<double> *__restrict__ in, cx<float> *__restrict__ out, int64_t m) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) out[i] = mk((float)in[i].re, (float)in[i].im);
}

// out = in for active right-hand sides, 0 for retired ones (FP64 -> FP32)
__global__ void k_to32_active(const cx<double> *__restrict__ in, cx<float> *__restrict__ out, int64_t len, int nrhs,
                              const int32_t *__restrict__ act) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= len * nrhs) return;
    out[i] = act[i / len] ? mk((float)in[i].re, (float)in[i].im) : mk(0.f, 0.f);
}

__global__ void k_to64(const cx<float> *__restrict__ in, cx<double> *__restrict__ out, int64_t m) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) out[i] = mk((double)in[i].re, (double)in[i].im);
}

// x += d (FP32 correction into the FP64 iterate)
__global__ void k_add_from32(cx<double> *__restrict__ x, const cx<float> *__restrict__ d, int64_t m) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) x[i] += mk((double)d[i].re, (double)d[i].im);
}

// the interior plans' self-triangle blocks, per scatterer
struct RegionCorr {
    const cx<double> *cv[MAXJ];
    const cx<double> *cg[MAXJ];
    const int32_t *tri_nodes[MAXJ];
    const int32_t *point_tri[MAXJ];
};

__global__ void k_precond_build(const double *__restrict__ nrm, const int32_t *__restrict__ point_tri,
                                const int32_t *__restrict__ tri_nodes, int m, const cx<double> *__restrict__ cv0,
                                const cx<double> *__restrict__ cg0, const RegionCorr C, const Regions R, int64_t n,
                                cx<double> *__restrict__ minv, int32_t *__restrict__ bad) {
    int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int32_t t = point_tri[a];
    int js = 0;
    for (int j = 0; j < m; ++j)
        if (tri_nodes[(int64_t)t * m + j] == (int32_t)a) js = j;
    // the node in its scatterer's plan
    const int rj = R.reg ? R.reg[a] : 0;
    const int64_t l = R.loc ? R.loc[a] : a;
    const int32_t tl = C.point_tri[rj][l];
    int jl = 0;
    for (int j = 0; j < m; ++j)
        if (C.tri_nodes[rj][(int64_t)tl * m + j] == (int32_t)l) jl = j;
    const cx<double> tc = R.tc[rj], gamma = R.gamma[rj];
    const double nv[3] = {nrm[3 * a], nrm[3 * a + 1], nrm[3 * a + 2]};
    cx<double> V0[3], V1[3];
    for (int i = 0; i < 3; ++i) {
        V0[i] = cv0[(a * m + js) * 3 + i];
        V1[i] = C.cv[rj][(l * m + jl) * 3 + i];
    }
    const cx<double> G0 = cg0[a * m + js], G1 = C.cg[rj][l * m + jl];
    cx<double> A[6][12];
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 12; ++j) A[i][j] = mk(0.0, 0.0);
    cx<double> nV0 = nv[0] * V0[0] + nv[1] * V0[1] + nv[2] * V0[2];
    cx<double> nV1 = nv[0] * V1[0] + nv[1] * V1[1] + nv[2] * V1[2];
    cx<double> K0[3][3], K1[3][3], T[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double d = i == j ? 1.0 : 0.0;
            K0[i][j] = nv[i] * V0[j] - d * nV0 - V0[i] * nv[j];
            K1[i][j] = nv[i] * V1[j] - d * nV1 - V1[i] * nv[j];
            T[i][j] = mk(d, 0.0) + (nv[i] * nv[j]) * tc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double d = i == j ? 1.0 : 0.0;
            A[i][j] = mk(0.5 * d, 0.0) + K0[i][j];
            A[i][3 + j] = d * (-G0);
            cx<double> kt = mk(0.0, 0.0);
            for (int q = 0; q < 3; ++q) kt += K1[i][q] * T[q][j];
            A[3 + i][j] = 0.5 * T[i][j] - kt;
            A[3 + i][3 + j] = d * (gamma * G1);
        }
    for (int i = 0; i < 6; ++i) A[i][6 + i] = mk(1.0, 0.0);
    // Gauss-Jordan with partial pivoting
    for (int c = 0; c < 6; ++c) {
        int piv = c;
        double best = abs2(A[c][c]);
        for (int r = c + 1; r < 6; ++r)
            if (abs2(A[r][c]) > best) {
                best = abs2(A[r][c]);
                piv = r;
            }
        if (!(best > 0.0)) {
            atomicOr(bad, 1);
            return;
        }
        if (piv != c)
            for (int j = 0; j < 12; ++j) {
                cx<double> tmp = A[c][j];
                A[c][j] = A[piv][j];
                A[piv][j] = tmp;
            }
        cx<double> inv = cdiv(mk(1.0, 0.0), A[c][c]);
        for (int j = 0; j < 12; ++j) A[c][j] = A[c][j] * inv;
        for (int r = 0; r < 6; ++r) {
            if (r == c) continue;
            cx<double> f = A[r][c];
            for (int j = 0; j < 12; ++j) A[r][j] -= f * A[c][j];
        }
    }
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) minv[a * 36 + i * 6 + j] = A[i][6 + j];
}

template <typename T>
__global__ void k_precond_apply(const cx<T> *__restrict__ minv, const cx<T> *__restrict__ v, cx<T> *__restrict__ z,
                                int64_t n, int nrhs) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const int64_t node = i % n;
    const cx<T> *M = minv + node * 36;
    const cx<T> *vi = v + i * 6;
    cx<T> in[6];
    for (int q = 0; q < 6; ++q) in[q] = vi[q];
    for (int r = 0; r < 6; ++r) {
        cx<T> s = mk(T(0), T(0));
        for (int q = 0; q < 6; ++q) s += M[r * 6 + q] * in[q];
        z[i * 6 + r] = s;
    }
}

// Inverse of every nb x nb block (nb = 3 or 6), Gauss-Jordan with partial
// pivoting in FP64: turns the stored M^{-1} back into M for the inner GMRES.
template <int NB>
__global__ void k_block_invert(const cx<double> *__restrict__ in, cx<double> *__restrict__ out, int64_t n,
                               int32_t *__restrict__ bad) {
    int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= n) return;
    cx<double> A[NB][2 * NB];
    for (int i = 0; i < NB; ++i)
        for (int j = 0; j < NB; ++j) {
            A[i][j] = in[(a * NB + i) * NB + j];
            A[i][NB + j] = mk(i == j ? 1.0 : 0.0, 0.0);
        }
    for (int c = 0; c < NB; ++c) {
        int piv = c;
        double best = abs2(A[c][c]);
        for (int r = c + 1; r < NB; ++r)
            if (abs2(A[r][c]) > best) {
                best = abs2(A[r][c]);
                piv = r;
            }
        if (!(best > 0.0)) {
            atomicOr(bad, 1);
            return;
        }
        if (piv != c)
            for (int j = 0; j < 2 * NB; ++j) {
                const cx<double> t = A[c][j];
                A[c][j] = A[piv][j];
                A[piv][j] = t;
            }
        const cx<double> inv = cdiv(mk(1.0, 0.0), A[c][c]);
        for (int j = 0; j < 2 * NB; ++j) A[c][j] = A[c][j] * inv;
        for (int r = 0; r < NB; ++r) {
            if (r == c) continue;
            const cx<double> f = A[r][c];
            for (int j = 0; j < 2 * NB; ++j) A[r][j] -= f * A[c][j];
        }
    }
    for (int i = 0; i < NB; ++i)
        for (int j = 0; j < NB; ++j) out[(a * NB + i) * NB + j] = A[i][NB + j];
}

// out = M v per node (herm = 1: M^H v) for [nrhs][n][nb] vectors
template <typename T>
__global__ void k_block_mul(const cx<T> *__restrict__ blk, int nb, int herm, const cx<T> *__restrict__ v,
                            cx<T> *__restrict__ out, int64_t n, int nrhs) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const cx<T> *M = blk + (i % n) * nb * nb;
    const cx<T> *vi = v + i * nb;
    for (int r = 0; r < nb; ++r) {
        cx<T> acc = mk(T(0), T(0));
        for (int q = 0; q < nb; ++q) acc += (herm ? conj(M[q * nb + r]) : M[r * nb + q]) * vi[q];
        out[i * nb + r] = acc;
    }
}

// z = M^{-1} v per node (the block preconditioner) and, in the same pass, the
// split of z into the densities of the two plans (as k_bem_split)
template <typename T>
__global__ void k_precond_split(const cx<T> *__restrict__ minv, const cx<T> *__restrict__ v, cx<T> *__restrict__ z,
                                const double *__restrict__ nrm, int64_t n, int nrhs, const Regions R,
                                cx<T> *__restrict__ a0, cx<T> *__restrict__ b0, cx<T> *__restrict__ a1,
                                cx<T> *__restrict__ b1) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const int64_t node = i % n;
    const cx<T> *M = minv + node * 36;
    const cx<T> *vi = v + i * 6;
    cx<T> in[6], x[6];
    for (int q = 0; q < 6; ++q) in[q] = vi[q];
    for (int r = 0; r < 6; ++r) {
        cx<T> s = mk(T(0), T(0));
        for (int q = 0; q < 6; ++q) s += M[r * 6 + q] * in[q];
        x[r] = s;
        z[i * 6 + r] = s;
    }
    int j;
    const int64_t ii = interior_at(R, i, n, j);
    const cx<T> tc = narrow<T>(R.tc[j]), gamma = narrow<T>(R.gamma[j]);
    const T nv[3] = {(T)nrm[3 * node], (T)nrm[3 * node + 1], (T)nrm[3 * node + 2]};
    const cx<T> d = nv[0] * x[0] + nv[1] * x[1] + nv[2] * x[2];
    for (int c = 0; c < 3; ++c) {
        a0[i * 3 + c] = x[c];
        b0[i * 3 + c] = -x[3 + c];
        a1[ii + c] = x[c] + (nv[c] * tc) * d;
        b1[ii + c] = -(gamma * x[3 + c]);
    }
}

// ---- the adjoint system A^H ----
// With x = (Phi, Psi) the rows of A are r0 = 1/2 Phi + Op0(Phi, -Psi) and
// r1 = 1/2 T Phi - Op1(T Phi, -gamma Psi), T = I + tc n n^T.  Hence, for v =
// (v0, v1) and (a_j, b_j) = Op_j^H v_j,
//   (A^H v)[0:3] = 1/2 v0 + a0 + 1/2 T^H v1 - T^H a1,
//   (A^H v)[3:6] = -b0 + conj(gamma) b1,          T^H u = u + conj(tc) n (n . u).
template <typename T>
__global__ void k_adj_split(const cx<T> *__restrict__ x, int64_t n, int nrhs, const Regions R,
                            cx<T> *__restrict__ y0, cx<T> *__restrict__ y1) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    int j;
    const int64_t ii = interior_at(R, i, n, j);
    for (int c = 0; c < 3; ++c) {
        y0[i * 3 + c] = x[i * 6 + c];
        y1[ii + c] = x[i * 6 + 3 + c];
    }
}

// z = M^{-H} v per node (conjugate transpose of the 6x6 block inverse), split as k_adj_split
template <typename T>
__global__ void k_adj_precond_split(const cx<T> *__restrict__ minv, const cx<T> *__restrict__ v,
                                    cx<T> *__restrict__ z, int64_t n, int nrhs, const Regions R,
                                    cx<T> *__restrict__ y0, cx<T> *__restrict__ y1) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const int64_t node = i % n;
    int j;
    const int64_t ii = interior_at(R, i, n, j);
    const cx<T> *M = minv + node * 36;
    const cx<T> *vi = v + i * 6;
    cx<T> in[6];
    for (int q = 0; q < 6; ++q) in[q] = vi[q];
    for (int r = 0; r < 6; ++r) {
        cx<T> acc = mk(T(0), T(0));
        for (int q = 0; q < 6; ++q) acc += conj(M[q * 6 + r]) * in[q];
        z[i * 6 + r] = acc;
        if (r < 3) y0[i * 3 + r] = acc;
        else y1[ii + r - 3] = acc;
    }
}

template <typename T>
__global__ void k_adj_combine(const cx<T> *__restrict__ x, const double *__restrict__ nrm, int64_t n, int nrhs,
                              const Regions R, const cx<T> *__restrict__ a0, const cx<T> *__restrict__ b0,
                              const cx<T> *__restrict__ a1, const cx<T> *__restrict__ b1, cx<T> *__restrict__ r) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const int64_t node = i % n;
    int j;
    const int64_t ii = interior_at(R, i, n, j);
    const cx<T> tch = narrow<T>(conj(R.tc[j])), gc = narrow<T>(conj(R.gamma[j]));
    const T nv[3] = {(T)nrm[3 * node], (T)nrm[3 * node + 1], (T)nrm[3 * node + 2]};
    const cx<T> *xi = x + i * 6;
    cx<T> u[3];                                        // 1/2 v1 - a1, then T^H of it
    for (int c = 0; c < 3; ++c) u[c] = T(0.5) * xi[3 + c] - a1[ii + c];
    const cx<T> d = nv[0] * u[0] + nv[1] * u[1] + nv[2] * u[2];
    for (int c = 0; c < 3; ++c) {
        r[i * 6 + c] = T(0.5) * xi[c] + a0[i * 3 + c] + u[c] + (nv[c] * tch) * d;
        r[i * 6 + 3 + c] = gc * b1[ii + c] - b0[i * 3 + c];
    }
}



__global__ void k_rhs_planewave(const double *__restrict__ spts, const int32_t *__restrict__ iperm,
                                const double *__restrict__ dirs, const cx<double> *__restrict__ pols, int64_t n, int nrhs,
                                double k_re, double k_im, int nu, cx<double> *__restrict__ rhs) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const int64_t node = i % n, q = i / n;
    const int64_t si = iperm[node];
    const double ph = dirs[3 * q] * spts[3 * si] + dirs[3 * q + 1] * spts[3 * si + 1] + dirs[3 * q + 2] * spts[3 * si + 2];
    // exp(i k ph) = exp(-k_im ph) (cos(k_re ph) + i sin(k_re ph))
    double s, c;
    sincos(k_re * ph, &s, &c);
    const double e = exp(-k_im * ph);
    const cx<double> w = mk(e * c, e * s);
    for (int d = 0; d < 3; ++d) rhs[i * nu + d] = pols[3 * q + d] * w;
    for (int d = 3; d < nu; ++d) rhs[i * nu + d] = mk(0.0, 0.0);
}

// ---- impedance boundary condition (eq. 2.25), three unknowns per node ----
//   A Phi = 1/2 Phi + Op0(Phi, c n x (n x Phi)),  n x (n x v) = n (n . v) - v,
//   A^H v = 1/2 v + a + conj(c) n x (n x b),  (a, b) = Op0^H v.
template <typename T>
__device__ inline void nnx(const T nv[3], const cx<T> in[3], cx<T> out[3]) {
    const cx<T> d = nv[0] * in[0] + nv[1] * in[1] + nv[2] * in[2];
    for (int q = 0; q < 3; ++q) out[q] = nv[q] * d - in[q];
}

// b = c n x (n x x); with minv, x is first set to M^{-1} v (3x3 blocks)
template <typename T>
__global__ void k_ibc_split(const cx<T> *__restrict__ minv, const cx<T> *__restrict__ v, cx<T> *__restrict__ x,
                            const double *__restrict__ nrm, int64_t n, int nrhs, cx<double> cd,
                            cx<T> *__restrict__ b) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const int64_t node = i % n;
    const T nv[3] = {(T)nrm[3 * node], (T)nrm[3 * node + 1], (T)nrm[3 * node + 2]};
    cx<T> xi[3];
    if (minv) {
        const cx<T> *M = minv + node * 9;
        for (int r = 0; r < 3; ++r) {
            cx<T> acc = mk(T(0), T(0));
            for (int q = 0; q < 3; ++q) acc += M[r * 3 + q] * v[i * 3 + q];
            xi[r] = acc;
        }
        for (int r = 0; r < 3; ++r) x[i * 3 + r] = xi[r];
    } else {
        for (int r = 0; r < 3; ++r) xi[r] = x[i * 3 + r];
    }
    cx<T> t[3];
    nnx(nv, xi, t);
    const cx<T> c = narrow<T>(cd);
    for (int q = 0; q < 3; ++q) b[i * 3 + q] = c * t[q];
}

template <typename T>
__global__ void k_ibc_combine(const cx<T> *__restrict__ x, const cx<T> *__restrict__ y0, int64_t m,
                              cx<T> *__restrict__ r) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) r[i] = T(0.5) * x[i] + y0[i];
}

// z = M^{-H} v (3x3 blocks)
template <typename T>
__global__ void k_ibc_adj_precond(const cx<T> *__restrict__ minv, const cx<T> *__restrict__ v, cx<T> *__restrict__ z,
                                  int64_t n, int nrhs) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const cx<T> *M = minv + (i % n) * 9;
    for (int r = 0; r < 3; ++r) {
        cx<T> acc = mk(T(0), T(0));
        for (int q = 0; q < 3; ++q) acc += conj(M[q * 3 + r]) * v[i * 3 + q];
        z[i * 3 + r] = acc;
    }
}

template <typename T>
__global__ void k_ibc_adj_combine(const cx<T> *__restrict__ x, const double *__restrict__ nrm, int64_t n, int nrhs,
                                  cx<double> cd, const cx<T> *__restrict__ a0, const cx<T> *__restrict__ b0,
                                  cx<T> *__restrict__ r) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n * nrhs) return;
    const int64_t node = i % n;
    const T nv[3] = {(T)nrm[3 * node], (T)nrm[3 * node + 1], (T)nrm[3 * node + 2]};
    cx<T> bb[3], t[3];
    for (int q = 0; q < 3; ++q) bb[q] = b0[i * 3 + q];
    nnx(nv, bb, t);
    const cx<T> ch = narrow<T>(conj(cd));
    for (int q = 0; q < 3; ++q) r[i * 3 + q] = T(0.5) * x[i * 3 + q] + a0[i * 3 + q] + ch * t[q];
}

// 3x3 preconditioner blocks 1/2 I + K(dV) + c dG (n n^T - I), inverted by Gauss-Jordan in FP64
__global__ void k_ibc_precond_build(const double *__restrict__ nrm, const int32_t *__restrict__ point_tri,
                                    const int32_t *__restrict__ tri_nodes, int m, const cx<double> *__restrict__ cv,
                                    const cx<double> *__restrict__ cg, int64_t n, cx<double> c,
                                    cx<double> *__restrict__ minv, int32_t *__restrict__ bad) {
    int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int32_t t = point_tri[a];
    int js = 0;
    for (int j = 0; j < m; ++j)
        if (tri_nodes[(int64_t)t * m + j] == (int32_t)a) js = j;
    const double nv[3] = {nrm[3 * a], nrm[3 * a + 1], nrm[3 * a + 2]};
    cx<double> V[3];
    for (int i = 0; i < 3; ++i) V[i] = cv[(a * m + js) * 3 + i];
    const cx<double> cG = c * cg[a * m + js];
    const cx<double> nV = nv[0] * V[0] + nv[1] * V[1] + nv[2] * V[2];
    cx<double> A[3][6];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double d = i == j ? 1.0 : 0.0;
            A[i][j] = mk(0.5 * d, 0.0) + nv[i] * V[j] - d * nV - V[i] * nv[j] + (nv[i] * nv[j] - d) * cG;
            A[i][3 + j] = mk(d, 0.0);
        }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        double best = abs2(A[col][col]);
        for (int r = col + 1; r < 3; ++r)
            if (abs2(A[r][col]) > best) {
                best = abs2(A[r][col]);
                piv = r;
            }
        if (!(best > 0.0)) {
            atomicOr(bad, 1);
            return;
        }
        if (piv != col)
            for (int j = 0; j < 6; ++j) {
                const cx<double> tmp = A[col][j];
                A[col][j] = A[piv][j];
                A[piv][j] = tmp;
            }
        const cx<double> inv = cdiv(mk(1.0, 0.0), A[col][col]);
        for (int j = 0; j < 6; ++j) A[col][j] = A[col][j] * inv;
        for (int r = 0; r < 3; ++r) {
            if (r == col) continue;
            const cx<double> f = A[r][col];
            for (int j = 0; j < 6; ++j) A[r][j] -= f * A[col][j];
        }
    }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) minv[a * 9 + i * 3 + j] = A[i][3 + j];
}

// ---- fields off the surface ----
// Eq. 2.5 at points off the boundary has the jump term 1 instead of 1/2, so in
// the row convention of the system the scattered field at host points is
// E_sca(r) = -Op_k0(a, b)(r) with a = Phi, b = -Psi (b = c n x (n x Phi) for the
// impedance condition), and the field inside the scatterer is
// E_1(r) = Op_k1(T Phi, -gamma Psi)(r), where
//   Op(a, b)(r) = sum_beta w_beta [ n (G . a) - (n . G) a - G (n . a) + g b ],
//   g = e^{ikR} / (4 pi R), G = grad' g = (ikR - 1) g (s_beta - r) / R^2.
// Far away E_sca ~ e^{ikr} / r F(rhat) with
//   F(rhat) = -(1/4pi) sum_beta w_beta e^{-ik rhat . s_beta} [ -ik (n (rhat . a) - (n . rhat) a - rhat (n . a)) + b ].
// Both are direct FP64 sums over all nodes: one thread per target point or
// direction, the nodes streamed through LDS in tiles.
constexpr int FE_TILE = 128;

struct FieldSrc {
    double pos[FE_TILE][3];
    double nrm[FE_TILE][3];
    double w[FE_TILE];
    cx<double> a[FE_TILE][3], b[FE_TILE][3];
};

// region: 0 host (scattered field), 1 interior; KIND 0: the field at points,
// 1: the far-field amplitude at unit directions, 2: curl of the scattered field
// at host points, -sum w [ Hess(g) c + k^2 g c + grad_r g x b ] with c = a x n
// (the summand's curl: its first term is grad_r g x c, the (n . a) grad_r g term
// is a gradient), grad_r g = g' u, Hess(g) = (g'' - g'/R) u u^T + (g'/R) I,
// u = (r - s)/R, g' = (ik - 1/R) g, g'' = ((ik - 1/R)^2 + 1/R^2) g.
template <int KIND>
__global__ void __launch_bounds__(FE_TILE) k_field(const double *__restrict__ tgt, int64_t nt,
                                                   const double *__restrict__ spts, const double *__restrict__ snrm,
                                                   const double *__restrict__ sw, const int32_t *__restrict__ perm,
                                                   const cx<double> *__restrict__ x, int64_t n, int nu, int region,
                                                   int ibc, double k_re, double k_im, cx<double> tc,
                                                   cx<double> gamma, cx<double> cibc, cx<double> *__restrict__ out) {
    __shared__ FieldSrc S;
    const int r = blockIdx.y;
    const int64_t t = blockIdx.x * (int64_t)FE_TILE + threadIdx.x;
    const bool active = t < nt;
    double p[3] = {0, 0, 0};
    if (active)
        for (int q = 0; q < 3; ++q) p[q] = tgt[3 * t + q];
    cx<double> acc[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
    const cx<double> k = mk(k_re, k_im);
    const double inv4pi = 0.07957747154594766788;
    for (int64_t base = 0; base < n; base += FE_TILE) {
        const int cnt = (int)min((int64_t)FE_TILE, n - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const int j = threadIdx.x;
            const int64_t i = base + j;
            const cx<double> *xi = x + ((int64_t)r * n + perm[i]) * nu;
            double nv[3];
            for (int q = 0; q < 3; ++q) {
                S.pos[j][q] = spts[3 * i + q];
                nv[q] = snrm[3 * i + q];
                S.nrm[j][q] = nv[q];
            }
            S.w[j] = sw[i];
            const cx<double> d = nv[0] * xi[0] + nv[1] * xi[1] + nv[2] * xi[2];
            for (int q = 0; q < 3; ++q) {
                if (ibc) {
                    S.a[j][q] = xi[q];
                    S.b[j][q] = cibc * (nv[q] * d - xi[q]);
                } else if (region == 0) {
                    S.a[j][q] = xi[q];
                    S.b[j][q] = -xi[3 + q];
                } else {
                    S.a[j][q] = xi[q] + (nv[q] * tc) * d;
                    S.b[j][q] = -(gamma * xi[3 + q]);
                }
            }
        }
        __syncthreads();
        if (!active) continue;
        for (int j = 0; j < cnt; ++j) {
            const double *nb = S.nrm[j];
            const cx<double> *a = S.a[j], *b = S.b[j];
            const cx<double> na = nb[0] * a[0] + nb[1] * a[1] + nb[2] * a[2];
            if (KIND == 2) {
                const double ux0 = p[0] - S.pos[j][0], uy0 = p[1] - S.pos[j][1], uz0 = p[2] - S.pos[j][2];
                const double R2 = ux0 * ux0 + uy0 * uy0 + uz0 * uz0;
                if (R2 <= 0.0) continue;
                const double R = sqrt(R2), iR = 1.0 / R;
                const double u[3] = {ux0 * iR, uy0 * iR, uz0 * iR};
                double sn, cs;
                sincos(k_re * R, &sn, &cs);
                const cx<double> g = (S.w[j] * inv4pi * iR * exp(-k_im * R)) * mk(cs, sn);
                const cx<double> ikr = mk(-k_im - iR, k_re);                  // i k - 1/R
                const cx<double> g1 = ikr * g;
                const cx<double> g2 = (ikr * ikr + mk(iR * iR, 0.0)) * g;
                const cx<double> c[3] = {a[1] * nb[2] - a[2] * nb[1], a[2] * nb[0] - a[0] * nb[2],
                                         a[0] * nb[1] - a[1] * nb[0]};
                const cx<double> uc = u[0] * c[0] + u[1] * c[1] + u[2] * c[2];
                const cx<double> hu = (g2 - iR * g1) * uc, hc = iR * g1, kk = k * k * g;
                const cx<double> gr[3] = {u[0] * g1, u[1] * g1, u[2] * g1};
                const cx<double> gxb[3] = {gr[1] * b[2] - gr[2] * b[1], gr[2] * b[0] - gr[0] * b[2],
                                           gr[0] * b[1] - gr[1] * b[0]};
                for (int q2 = 0; q2 < 3; ++q2) acc[q2] += u[q2] * hu + (hc + kk) * c[q2] + gxb[q2];
            } else if (KIND == 1) {
                // e^{-ik rhat . s} w / (4 pi) times [ -ik (n (rhat . a) - (n . rhat) a - rhat (n . a)) + b ]
                const double ph = p[0] * S.pos[j][0] + p[1] * S.pos[j][1] + p[2] * S.pos[j][2];
                double sn, cs;
                sincos(-k_re * ph, &sn, &cs);
                const cx<double> e = (S.w[j] * inv4pi * exp(k_im * ph)) * mk(cs, sn);
                const cx<double> ra = p[0] * a[0] + p[1] * a[1] + p[2] * a[2];
                const double nr = nb[0] * p[0] + nb[1] * p[1] + nb[2] * p[2];
                const cx<double> mik = mk(k_im, -k_re);           // -i k
                for (int q = 0; q < 3; ++q)
                    acc[q] += e * (mik * (nb[q] * ra - nr * a[q] - p[q] * na) + b[q]);
            } else {
                const double dx = S.pos[j][0] - p[0], dy = S.pos[j][1] - p[1], dz = S.pos[j][2] - p[2];
                const double R2 = dx * dx + dy * dy + dz * dz;
                if (R2 <= 0.0) continue;
                const double R = sqrt(R2), iR = 1.0 / R;
                double sn, cs;
                sincos(k_re * R, &sn, &cs);
                const cx<double> g = (S.w[j] * inv4pi * iR * exp(-k_im * R)) * mk(cs, sn);
                const cx<double> f = (iR * iR) * (mk(-k_im * R - 1.0, k_re * R) * g);
                const double dv[3] = {dx, dy, dz};
                const cx<double> Ga = dx * a[0] + dy * a[1] + dz * a[2];
                const double nG = nb[0] * dx + nb[1] * dy + nb[2] * dz;
                for (int q = 0; q < 3; ++q) acc[q] += f * (nb[q] * Ga - nG * a[q] - dv[q] * na) + g * b[q];
            }
        }
    }
    if (!active) return;
    const double sg = KIND != 0 ? -1.0 : (region == 0 ? -1.0 : 1.0);
    for (int q = 0; q < 3; ++q) out[((int64_t)r * nt + t) * 3 + q] = sg * acc[q];
}

// Conjugate transpose of the far-field map x -> F of k_field<1>.  With
// F(rhat) = sum_beta c [ M a_beta + b_beta ], c = -w e^{-ik rhat . s} / (4 pi) and
// M = -ik (n rhat^T - (n . rhat) I - rhat n^T), the adjoint of samples G(rhat) is
//   a_bar = sum_rhat conj(c) i conj(k) [ rhat (n . G) - (n . rhat) G - n (rhat . G) ],
//   b_bar = sum_rhat conj(c) G,
// then Phi_bar = a_bar, Psi_bar = -b_bar (dielectric), or for an impedance
// problem (b = c_Z (n n^T - I) Phi) Phi_bar = a_bar + conj(c_Z) (n (n . b_bar) - b_bar).
// One thread per node (sorted index), directions staged through LDS.
struct FarAdjTile {
    double dir[FE_TILE][3];
    cx<double> g[FE_TILE][3];
};

__global__ void __launch_bounds__(FE_TILE) k_far_adjoint(const double *__restrict__ dirs, int64_t nd,
                                                         const cx<double> *__restrict__ G,
                                                         const double *__restrict__ spts,
                                                         const double *__restrict__ snrm,
                                                         const double *__restrict__ sw,
                                                         const int32_t *__restrict__ perm, int64_t n, int nu, int ibc,
                                                         double k_re, double k_im, cx<double> cibc,
                                                         cx<double> *__restrict__ xbar) {
    __shared__ FarAdjTile S;
    const int r = blockIdx.y;
    const int64_t i = blockIdx.x * (int64_t)FE_TILE + threadIdx.x;
    const bool active = i < n;
    double s[3] = {0, 0, 0}, nv[3] = {0, 0, 0};
    if (active)
        for (int q = 0; q < 3; ++q) {
            s[q] = spts[3 * i + q];
            nv[q] = snrm[3 * i + q];
        }
    cx<double> aa[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
    cx<double> bb[3] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
    for (int64_t base = 0; base < nd; base += FE_TILE) {
        const int cnt = (int)min((int64_t)FE_TILE, nd - base);
        __syncthreads();
        if ((int)threadIdx.x < cnt) {
            const int64_t d = base + threadIdx.x;
            for (int q = 0; q < 3; ++q) {
                S.dir[threadIdx.x][q] = dirs[3 * d + q];
                S.g[threadIdx.x][q] = G[((int64_t)r * nd + d) * 3 + q];
            }
        }
        __syncthreads();
        if (!active) continue;
        for (int j = 0; j < cnt; ++j) {
            const double *u = S.dir[j];
            const cx<double> *g = S.g[j];
            const double ph = u[0] * s[0] + u[1] * s[1] + u[2] * s[2];
            double sn, cs;
            sincos(k_re * ph, &sn, &cs);
            const cx<double> ec = exp(k_im * ph) * mk(cs, sn);        // conj(e^{-ik rhat . s})
            const cx<double> nG = nv[0] * g[0] + nv[1] * g[1] + nv[2] * g[2];
            const cx<double> uG = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
            const double nu_ = nv[0] * u[0] + nv[1] * u[1] + nv[2] * u[2];
            for (int q = 0; q < 3; ++q) {
                aa[q] += ec * (u[q] * nG - nu_ * g[q] - nv[q] * uG);
                bb[q] += ec * g[q];
            }
        }
    }
    if (!active) return;
    const double fac = -sw[i] * 0.07957747154594766788;           // -w / (4 pi)
    const cx<double> ick = mk(k_im, k_re);                          // i conj(k)
    cx<double> *o = xbar + ((int64_t)r * n + perm[i]) * nu;
    if (ibc) {
        const cx<double> nb = nv[0] * bb[0] + nv[1] * bb[1] + nv[2] * bb[2];
        const cx<double> cz = mk(cibc.re, -cibc.im);
        for (int q = 0; q < 3; ++q) o[q] = fac * (ick * aa[q] + cz * (nv[q] * nb - bb[q]));
    } else {
        for (int q = 0; q < 3; ++q) {
            o[q] = fac * (ick * aa[q]);
            o[3 + q] = -(fac * bb[q]);
        }
    }
}

// Densities of the field sum laid out for a plan over the nodes (user order)
// followed by nt target points, zero at the targets: a = Phi, b = -Psi (host
// region), a = T Phi, b = -gamma Psi (interior), a = Phi, b = c n x (n x Phi)
// (impedance).  Threads run over the sorted node index and the targets.
__global__ void __launch_bounds__(TPB) k_field_dens(const double *__restrict__ snrm, const int32_t *__restrict__ perm,
                                                    const cx<double> *__restrict__ x, int64_t n, int64_t nt, int nu,
                                                    int region, int ibc, cx<double> tc, cx<double> gamma,
                                                    cx<double> cibc, cx<double> *__restrict__ a,
                                                    cx<double> *__restrict__ b) {
    const int r = blockIdx.y;
    const int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
    const int64_t m = n + nt;
    if (i >= m) return;
    cx<double> *ar = a + (int64_t)r * m * 3, *br = b + (int64_t)r * m * 3;
    if (i >= n) {
        for (int q = 0; q < 3; ++q) ar[3 * i + q] = br[3 * i + q] = mk(0.0, 0.0);
        return;
    }
    const int64_t u = perm[i];
    const cx<double> *xi = x + ((int64_t)r * n + u) * nu;
    const double nv[3] = {snrm[3 * i], snrm[3 * i + 1], snrm[3 * i + 2]};
    const cx<double> d = nv[0] * xi[0] + nv[1] * xi[1] + nv[2] * xi[2];
    for (int q = 0; q < 3; ++q) {
        cx<double> av, bv;
        if (ibc) {
            av = xi[q];
            bv = cibc * (nv[q] * d - xi[q]);
        } else if (region == 0) {
            av = xi[q];
            bv = -xi[3 + q];
        } else {
            av = xi[q] + (nv[q] * tc) * d;
            bv = -(gamma * xi[3 + q]);
        }
        ar[3 * u + q] = av;
        br[3 * u + q] = bv;
    }
}

// E[r][t] = sg * y[r][n + t]
__global__ void __launch_bounds__(TPB) k_field_take(const cx<double> *__restrict__ y, int64_t n, int64_t nt, double sg,
                                                    cx<double> *__restrict__ E) {
    const int r = blockIdx.y;
    const int64_t t = blockIdx.x * (int64_t)TPB + threadIdx.x;
    if (t >= nt) return;
    const cx<double> *yr = y + ((int64_t)r * (n + nt) + n + t) * 3;
    for (int q = 0; q < 3; ++q) E[((int64_t)r * nt + t) * 3 + q] = sg * yr[q];
}

// ---- Krylov kernels (vectors of length len per rhs, stride len) ----
// Vectors are cx<T> (T = double for FP64 solves, float for the inner solves of
// the mixed mode); inner products, the Hessenberg matrix and the rotations are
// always FP64.
constexpr int DOT_CHUNKS = 64;            // blocks per (vector, rhs) in the inner-product kernel

inline int nchunks_c(int64_t len) { return (int)((len + TPB - 1) / TPB); }   // update-kernel blocks per rhs
__device__ inline int nchunks_c_dev(int64_t len) { return (int)((len + TPB - 1) / TPB); }

__device__ inline cx<double> shfl_xor_cx(cx<double> v, int m) {
    return mk(__shfl_xor(v.re, m), __shfl_xor(v.im, m));
}

// sum of v over the block (TPB threads), fixed reduction order; result valid in thread 0
__device__ inline cx<double> block_sum(cx<double> v, cx<double> *sm) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += shfl_xor_cx(v, o);
    if (lane == 0) sm[wave] = v;
    __syncthreads();
    cx<double> s = sm[0];
    for (int w = 1; w < TPB / 64; ++w) s += sm[w];
    return s;
}

// part[(i*nrhs + r)*DOT_CHUNKS + c] = sum over chunk c of conj(V_i[r]) W[r] for
// i < nv, and for i == nv (when X is given) the same with X in place of V_i.
// need (optional): rhs with need[r] == 0 write zeros without reading.
template <typename T>
__global__ void __launch_bounds__(TPB) k_dots(const cx<T> *__restrict__ V, int64_t vstride, int nv,
                                              const cx<T> *__restrict__ X, const cx<T> *__restrict__ W, int64_t len,
                                              int nrhs, const int32_t *__restrict__ need,
                                              cx<double> *__restrict__ part) {
    __shared__ cx<double> sm[TPB / 64];
    const int c = blockIdx.x % DOT_CHUNKS;
    const int r = (blockIdx.x / DOT_CHUNKS) % nrhs;
    const int i = blockIdx.x / (DOT_CHUNKS * nrhs);
    cx<double> *out = part + ((int64_t)i * nrhs + r) * DOT_CHUNKS + c;
    if (need && !need[r]) {
        if (threadIdx.x == 0) *out = mk(0.0, 0.0);
        return;
    }
    const cx<T> *v = (i < nv ? V + (int64_t)i * vstride : X) + (int64_t)r * len;
    const cx<T> *w = W + (int64_t)r * len;
    const int64_t per = (len + DOT_CHUNKS - 1) / DOT_CHUNKS;
    const int64_t k0 = c * per, k1 = min(len, k0 + per);
    cx<double> s = mk(0.0, 0.0);
#pragma unroll 4
    for (int64_t k = k0 + threadIdx.x; k < k1; k += TPB) s += conj(widen(v[k])) * widen(w[k]);
    s = block_sum(s, sm);
    if (threadIdx.x == 0) *out = s;
}

// out[e] = sum_c part[e*DOT_CHUNKS + c], one wave per e (fixed order)
__global__ void k_dots_reduce(const cx<double> *__restrict__ part, int cnt, cx<double> *__restrict__ out) {
    const int e = blockIdx.x;
    if (e >= cnt) return;
    cx<double> s = part[(int64_t)e * DOT_CHUNKS + threadIdx.x];
    for (int o = 32; o > 0; o >>= 1) s += shfl_xor_cx(s, o);
    if (threadIdx.x == 0) out[e] = s;
}

// W[r] += sign * sum_i V_i[r] h[i][r]   (h laid out [i][nrhs]) for the rhs with
// active[r] (and need[r]); with npart, also each block's |W_new|^2 into
// npart[r*nchunks_c(len) + block].  One element per thread; blocks do not
// straddle rhs; h of the block's rhs in LDS.
template <typename T>
__global__ void __launch_bounds__(TPB) k_combine(const cx<T> *__restrict__ V, int64_t vstride, int nv,
                                                 const cx<double> *__restrict__ h, double sign,
                                                 cx<T> *__restrict__ W, int64_t len, int nrhs,
                                                 const int32_t *__restrict__ active,
                                                 const int32_t *__restrict__ need, double *__restrict__ npart) {
    extern __shared__ cx<double> sh[];                 // [nv]
    __shared__ cx<double> sm[TPB / 64];
    const int nb = nchunks_c_dev(len);
    const int c = blockIdx.x % nb, r = blockIdx.x / nb;
    if ((active && !active[r]) || (need && !need[r])) {
        if (npart && threadIdx.x == 0) npart[(int64_t)r * nb + c] = 0.0;
        return;
    }
    for (int i = threadIdx.x; i < nv; i += TPB) sh[i] = sign * h[(int64_t)i * nrhs + r];
    __syncthreads();
    const int64_t k = (int64_t)c * TPB + threadIdx.x;
    double n2 = 0.0;
    if (k < len) {
        const int64_t e = (int64_t)r * len + k;
        cx<double> acc = widen(W[e]);
#pragma unroll 8
        for (int i = 0; i < nv; ++i) acc += widen(V[(int64_t)i * vstride + e]) * sh[i];
        const cx<T> o = narrow<T>(acc);
        W[e] = o;
        n2 = abs2(widen(o));
    }
    if (npart) {
        const cx<double> t = block_sum(mk(n2, 0.0), sm);
        if (threadIdx.x == 0) npart[(int64_t)r * nb + c] = t.re;
    }
}

// After the first Gram-Schmidt pass: hn = |W'| from the chunk partials, and the
// Daniel-Gragg-Kaufman-Stewart test for a second pass, taken when the first
// one removed more than half of |A z|^2 = h[j+1] (|W'|^2 < |A z|^2 / 2).
// One wave per rhs.
__global__ void k_post1(const double *__restrict__ npart, int nch, const cx<double> *__restrict__ h, int j,
                        const int32_t *__restrict__ active, int32_t *__restrict__ need, double *__restrict__ hn,
                        double *__restrict__ hninv, int nrhs) {
    const int r = blockIdx.x;
    double s = 0.0;
    for (int c = threadIdx.x; c < nch; c += 64) s += npart[(int64_t)r * nch + c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (threadIdx.x == 0) {
        const double v = sqrt(s);
        hn[r] = v;
        hninv[r] = v > 0 ? 1.0 / v : 0.0;
        need[r] = (active[r] && 2.0 * s < h[(int64_t)(j + 1) * nrhs + r].re) ? 1 : 0;
    }
}

// After the second pass (rhs with need[r]): h += h2 and, the basis being
// orthonormal, |W''|^2 = |W'|^2 - |h2|^2.  One wave per rhs.
__global__ void k_post2(cx<double> *__restrict__ h, const cx<double> *__restrict__ h2, int nv,
                        const int32_t *__restrict__ need, double *__restrict__ hn, double *__restrict__ hninv,
                        int nrhs) {
    const int r = blockIdx.x;
    if (!need[r]) return;
    double s = 0.0;
    for (int i = threadIdx.x; i < nv; i += 64) {
        const cx<double> d = h2[(int64_t)i * nrhs + r];
        h[(int64_t)i * nrhs + r] += d;
        s += abs2(d);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (threadIdx.x == 0) {
        const double v = sqrt(fmax(hn[r] * hn[r] - s, 0.0));
        hn[r] = v;
        hninv[r] = v > 0 ? 1.0 / v : 0.0;
    }
}

template <typename T>
__global__ void k_scale_into(const cx<T> *__restrict__ W, const double *__restrict__ inv, cx<T> *__restrict__ out,
                             int64_t len, int nrhs, const int32_t *__restrict__ active) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= len * nrhs) return;
    const int r = (int)(e / len);
    out[e] = (active && !active[r]) ? mk(T(0), T(0)) : narrow<T>(inv[r] * widen(W[e]));
}

template <typename T>
__global__ void k_sub(const cx<T> *__restrict__ b, const cx<T> *__restrict__ ax, cx<T> *__restrict__ r, int64_t m) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < m) r[i] = b[i] - ax[i];
}

// One Arnoldi column per rhs (one block each): H[:, j] from h (j+1 entries,
// [i][nrhs]) and hn; apply the old rotations, form a new one, update g, write
// the residual estimate.  |A z| (for the breakdown test) is sqrt of h[j+1] =
// (A z)^H (A z), the extra inner product of the first Gram-Schmidt pass.  The
// column and the rotations are staged in LDS; one thread applies them in order.
// The residual estimate and the breakdown flag go straight to host-mapped
// memory (hres, hbrk), and a rhs whose estimate reached tol |b| (bnd) or that
// broke down is retired here (active = 0); the host applies the same rule to
// the same values.
__global__ void k_givens(cx<double> *__restrict__ H, int ldh, int j, const cx<double> *__restrict__ h,
                         const double *__restrict__ hn, double *__restrict__ cs, cx<double> *__restrict__ sn,
                         cx<double> *__restrict__ g, int32_t *__restrict__ active, const double *__restrict__ bnd,
                         double tol, double *__restrict__ hres, int32_t *__restrict__ hbrk, int nrhs, int m) {
    extern __shared__ unsigned char gsm[];
    cx<double> *col = reinterpret_cast<cx<double> *>(gsm);          // [j+2]
    cx<double> *ssn = col + (j + 2);                                 // [j]
    double *scs = reinterpret_cast<double *>(ssn + j);               // [j]
    const int r = blockIdx.x;
    if (!active[r]) return;
    for (int i = threadIdx.x; i <= j; i += blockDim.x) col[i] = h[(int64_t)i * nrhs + r];
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
        scs[i] = cs[r * m + i];
        ssn[i] = sn[r * m + i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double nAz = sqrt(fmax(h[(int64_t)(j + 1) * nrhs + r].re, 0.0));
        col[j + 1] = mk(hn[r], 0.0);
        for (int i = 0; i < j; ++i) {
            const double c = scs[i];
            const cx<double> s = ssn[i];
            cx<double> t = c * col[i] + s * col[i + 1];
            col[i + 1] = c * col[i + 1] - conj(s) * col[i];
            col[i] = t;
        }
        const cx<double> a = col[j], b = col[j + 1];
        const double aa = sqrt(abs2(a)), den = sqrt(abs2(a) + abs2(b));
        double c;
        cx<double> s;
        if (aa == 0.0) {
            c = 0.0;
            s = mk(1.0, 0.0);
        } else {
            c = aa / den;
            s = (1.0 / (aa * den)) * (a * conj(b));
        }
        cs[r * m + j] = c;
        sn[r * m + j] = s;
        col[j] = c * a + s * b;
        col[j + 1] = mk(0.0, 0.0);
        cx<double> gj = g[r * (m + 1) + j];
        g[r * (m + 1) + j + 1] = -(conj(s) * gj);
        g[r * (m + 1) + j] = c * gj;
        const double res = sqrt(abs2(g[r * (m + 1) + j + 1]));
        const int32_t brk = (hn[r] <= 1e-14 * nAz) ? 1 : 0;
        hres[r] = res;
        hbrk[r] = brk;
        if (res <= tol * bnd[r] || brk) active[r] = 0;
    }
    __syncthreads();
    cx<double> *Hc = H + (int64_t)r * ldh * m + (int64_t)j * ldh;   // column-major [m][ldh]
    for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) Hc[i] = col[i];
}

// y = H^{-1} g (upper triangular, size jr[r]) per rhs, written as y[i][nrhs]
__global__ void k_trisolve(const cx<double> *__restrict__ H, int ldh, const cx<double> *__restrict__ g,
                           const int32_t *__restrict__ jr, cx<double> *__restrict__ y, int nrhs, int m) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    const cx<double> *Hr = H + (int64_t)r * ldh * m;
    const int J = jr[r];
    for (int i = 0; i < m; ++i) y[(int64_t)i * nrhs + r] = mk(0.0, 0.0);
    for (int i = J - 1; i >= 0; --i) {
        cx<double> s = g[r * (m + 1) + i];
        for (int q = i + 1; q < J; ++q) s -= Hr[(int64_t)q * ldh + i] * y[(int64_t)q * nrhs + r];
        y[(int64_t)i * nrhs + r] = cdiv(s, Hr[(int64_t)i * ldh + i]);
    }
}

// out = sqrt(re in), inv = 1/out (0 for 0)
__global__ void k_sqrt_real(const cx<double> *__restrict__ in, double *__restrict__ out, double *__restrict__ inv,
                            int m) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double v = sqrt(fmax(in[i].re, 0.0));
    out[i] = v;
    if (inv) inv[i] = v > 0 ? 1.0 / v : 0.0;
}

// host memory the device writes directly (allocated pinned and mapped)
struct HostMapped {
    void *h = nullptr, *d = nullptr;
    HostMapped() = default;
    HostMapped(const HostMapped &) = delete;
    HostMapped &operator=(const HostMapped &) = delete;
    void alloc(size_t bytes) {
        release();
        FMB_CHECK_HIP(hipHostMalloc(&h, bytes, hipHostMallocMapped));
        FMB_CHECK_HIP(hipHostGetDevicePointer(&d, h, 0));
    }
    void release() {
        if (h) (void)hipHostFree(h);
        h = d = nullptr;
    }
    ~HostMapped() { release(); }
};

template <typename T>
struct Krylov {
    int64_t len = 0;
    int nrhs = 0, m = 0, nchc = 0;
    HostMapped step;   // two slots (step parity) of: double res[nrhs], int32 brk[nrhs]
    DevBuf bnd;        // |b| per rhs (device copy of the values the host holds)
    hipEvent_t ev[2] = {nullptr, nullptr};   // recorded after the Givens step, per slot
    Krylov() = default;
    Krylov(const Krylov &) = delete;
    Krylov &operator=(const Krylov &) = delete;
    ~Krylov() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    DevBuf V, Z, W, r, ax;                                            // cx<T>
    DevBuf H, cs, sn, g, h, h2, hn, hninv, part, npart, act, jr, y, tmp, need;   // FP64 / int32
};

// out[i][r] = V_i[r]^H W[r] for i < nv, plus X[r]^H W[r] as entry nv when X is given
template <typename T>
void dots(Krylov<T> &K, const cx<T> *V, int nv, const cx<T> *X, const cx<T> *W, const int32_t *need, cx<double> *out,
          hipStream_t s) {
    const int nvt = nv + (X ? 1 : 0);
    k_dots<T><<<(unsigned)(nvt * K.nrhs * DOT_CHUNKS), TPB, 0, s>>>(V, K.len * K.nrhs, nv, X, W, K.len, K.nrhs,
                                                                    need, K.part.template as<cx<double>>());
    k_dots_reduce<<<nvt * K.nrhs, 64, 0, s>>>(K.part.template as<cx<double>>(), nvt * K.nrhs, out);
    FMB_LAUNCH_CHECK();
}

template <typename T>
void norms(Krylov<T> &K, const cx<T> *W, double *out, double *inv, hipStream_t s) {
    dots(K, W, 1, (const cx<T> *)nullptr, W, (const int32_t *)nullptr, K.tmp.template as<cx<double>>(), s);
    k_sqrt_real<<<1, 1024, 0, s>>>(K.tmp.template as<cx<double>>(), out, inv, K.nrhs);
    FMB_LAUNCH_CHECK();
}

// W -= V h (sign -1) or W += V h (sign +1) over nv vectors
template <typename T>
void combine(Krylov<T> &K, const cx<T> *V, int nv, const cx<double> *h, double sign, cx<T> *W, const int32_t *active,
             const int32_t *need, double *npart, hipStream_t s) {
    k_combine<T><<<(unsigned)(K.nchc * K.nrhs), TPB, (size_t)std::max(nv, 1) * sizeof(cx<double>), s>>>(
        V, K.len * K.nrhs, nv, h, sign, W, K.len, K.nrhs, active, need, npart);
    FMB_LAUNCH_CHECK();
}

template <typename T>
void krylov_alloc(Krylov<T> &K, int64_t len, int nrhs, int m) {
    if (K.len == len && K.nrhs == nrhs && K.m == m) return;
    K.len = len;
    K.nrhs = nrhs;
    K.m = m;
    K.nchc = nchunks_c(len);
    const size_t tot = (size_t)len * nrhs * sizeof(cx<T>);
    K.V.alloc(tot * (m + 1));
    K.Z.alloc(tot * m);
    K.W.alloc(tot);
    K.r.alloc(tot);
    K.ax.alloc(tot);
    K.H.alloc((size_t)nrhs * (m + 1) * m * sizeof(cx<double>));
    K.cs.alloc((size_t)nrhs * m * sizeof(double));
    K.sn.alloc((size_t)nrhs * m * sizeof(cx<double>));
    K.g.alloc((size_t)nrhs * (m + 1) * sizeof(cx<double>));
    K.h.alloc((size_t)(m + 2) * nrhs * sizeof(cx<double>));
    K.h2.alloc((size_t)(m + 2) * nrhs * sizeof(cx<double>));
    K.y.alloc((size_t)(m + 1) * nrhs * sizeof(cx<double>));
    K.hn.alloc(nrhs * sizeof(double));
    K.hninv.alloc(nrhs * sizeof(double));
    K.act.alloc(nrhs * sizeof(int32_t));
    K.jr.alloc(nrhs * sizeof(int32_t));
    K.need.alloc(nrhs * sizeof(int32_t));
    K.tmp.alloc((size_t)(m + 2) * nrhs * sizeof(cx<double>));
    K.part.alloc((size_t)(m + 2) * nrhs * DOT_CHUNKS * sizeof(cx<double>));
    K.npart.alloc((size_t)nrhs * K.nchc * sizeof(double));
    K.bnd.alloc(nrhs * sizeof(double));
    K.step.alloc((size_t)2 * nrhs * (sizeof(double) + sizeof(int32_t)));
    for (hipEvent_t &e : K.ev)
        if (!e) FMB_CHECK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
}

}  // namespace

// The two FMM products of one BEM application run concurrently: the k1 plan
// on the problem's second stream, forked from and joined back into s.
template <typename T>
static void fmm_pair_eager(fmb_problem_s &pb, const Plan *P0, const Plan *P1, const cx<T> *a0, const cx<T> *b0,
                           cx<T> *y0, const cx<T> *a1, const cx<T> *b1, cx<T> *y1, int nrhs, hipStream_t s) {
    if (pb.serial) {
        run_matvec(*const_cast<Plan *>(P0), a0, b0, y0, nrhs, s);
        run_matvec(*const_cast<Plan *>(P1), a1, b1, y1, nrhs, s);
        return;
    }
    FMB_CHECK_HIP(hipEventRecord(pb.ev_fork, s));
    FMB_CHECK_HIP(hipStreamWaitEvent(pb.s2, pb.ev_fork, 0));
    run_matvec_pair(*const_cast<Plan *>(P0), a0, b0, y0, s, *const_cast<Plan *>(P1), a1, b1, y1, pb.s2, nrhs);
    FMB_CHECK_HIP(hipEventRecord(pb.ev_join, pb.s2));
    FMB_CHECK_HIP(hipStreamWaitEvent(s, pb.ev_join, 0));
}

// The two products, replayed from a captured graph (one launch instead of
// some fifty) unless graphs are off or a plan's stage timers are on.
template <typename T>
static void fmm_pair(fmb_problem_s &pb, const Plan *P0, const Plan *P1, const cx<T> *a0, const cx<T> *b0, cx<T> *y0,
                     const cx<T> *a1, const cx<T> *b1, cx<T> *y1, int nrhs, hipStream_t s) {
    if (!pb.graphs || P0->timer.mask || P1->timer.mask) {
        fmm_pair_eager<T>(pb, P0, P1, a0, b0, y0, a1, b1, y1, nrhs, s);
        return;
    }
    fmb_problem_s::PairGraph &G = sizeof(T) == sizeof(float) ? pb.g32 : pb.g64;
    FMB_CHECK_HIP(hipEventRecord(pb.ev_in, s));
    FMB_CHECK_HIP(hipStreamWaitEvent(pb.s1, pb.ev_in, 0));
    if (!G.exec || G.nrhs != nrhs || G.serial != pb.serial) {
        if (G.exec) FMB_CHECK_HIP(hipGraphExecDestroy(G.exec));
        G.exec = nullptr;
        FMB_CHECK_HIP(hipStreamBeginCapture(pb.s1, hipStreamCaptureModeThreadLocal));
        hipGraph_t graph = nullptr;
        try {
            fmm_pair_eager<T>(pb, P0, P1, a0, b0, y0, a1, b1, y1, nrhs, pb.s1);
        } catch (...) {
            (void)hipStreamEndCapture(pb.s1, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        FMB_CHECK_HIP(hipStreamEndCapture(pb.s1, &graph));
        const hipError_t e = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        FMB_CHECK_HIP(e);
        G.nrhs = nrhs;
        G.serial = pb.serial;
    }
    FMB_CHECK_HIP(hipGraphLaunch(G.exec, pb.s1));
    FMB_CHECK_HIP(hipEventRecord(pb.ev_out, pb.s1));
    FMB_CHECK_HIP(hipStreamWaitEvent(s, pb.ev_out, 0));
}

// The two adjoint products of an application: P0 on s and P1 on the
// problem's second stream (or both on s when the problem runs serially).
static void adjoint_pair(fmb_problem_s &pb, Plan &P0, Plan &P1, const void *y0, void *a0, void *b0, const void *y1,
                         void *a1, void *b1, int nrhs, hipStream_t s) {
    if (pb.serial) {
        run_matvec_adjoint(P0, y0, a0, b0, nrhs, s);
        run_matvec_adjoint(P1, y1, a1, b1, nrhs, s);
        return;
    }
    adjoint_prepare(P0);
    adjoint_prepare(P1);
    FMB_CHECK_HIP(hipEventRecord(pb.ev_fork, s));
    FMB_CHECK_HIP(hipStreamWaitEvent(pb.s2, pb.ev_fork, 0));
    run_matvec_adjoint(P0, y0, a0, b0, nrhs, s);
    run_matvec_adjoint(P1, y1, a1, b1, nrhs, pb.s2);
    FMB_CHECK_HIP(hipEventRecord(pb.ev_join, pb.s2));
    FMB_CHECK_HIP(hipStreamWaitEvent(s, pb.ev_join, 0));
}

// The products of a several-scatterer application: the host plan on s, the
// scatterers' plans one after the other on the problem's second stream (all on
// s when the problem runs serially).  Forward: (in0, in0b) -> out0 with the host
// plan and (in1, in1b) -> out1 blockwise; adjoint: in0 -> (out0a, out0b) and
// in1 -> (out1a, out1b).  Block j of the interior arrays starts at off[j].
template <typename T>
static void multi_products(fmb_problem_s &pb, bool adj, const cx<T> *u0, cx<T> *v0, cx<T> *w0, const cx<T> *u1,
                           cx<T> *v1, cx<T> *w1, int nrhs, hipStream_t s) {
    const bool f32 = sizeof(T) == sizeof(float);
    Plan &P0 = f32 ? pb.p032->p : pb.p0->p;
    hipStream_t s2 = pb.serial ? s : pb.s2;
    if (adj) {
        adjoint_prepare(P0);
        for (int j = 0; j < pb.J; ++j) adjoint_prepare(f32 ? pb.pj32[j]->p : pb.pj[j]->p);
    }
    if (!pb.serial) {
        FMB_CHECK_HIP(hipEventRecord(pb.ev_fork, s));
        FMB_CHECK_HIP(hipStreamWaitEvent(s2, pb.ev_fork, 0));
    }
    // forward: (u, v) -> w;  adjoint: u -> (v, w)
    if (adj) run_matvec_adjoint(P0, u0, v0, w0, nrhs, s);
    else run_matvec(P0, u0, v0, w0, nrhs, s);
    for (int j = 0; j < pb.J; ++j) {
        Plan &Pj = f32 ? pb.pj32[j]->p : pb.pj[j]->p;
        const int64_t o = pb.off[j];
        if (adj) run_matvec_adjoint(Pj, u1 + o, v1 + o, w1 + o, nrhs, s2);
        else run_matvec(Pj, u1 + o, v1 + o, w1 + o, nrhs, s2);
    }
    if (!pb.serial) {
        FMB_CHECK_HIP(hipEventRecord(pb.ev_join, s2));
        FMB_CHECK_HIP(hipStreamWaitEvent(s, pb.ev_join, 0));
    }
}

// The impedance-boundary-condition system: A x (or A^H x in adjoint mode)
// with the k0 plan alone; with pre = v, x is first set to M^{-1} v (M^{-H} v).
template <typename T>
static void ibc_apply_t(fmb_problem_s &pb, const cx<T> *x, cx<T> *r, int nrhs, hipStream_t s, const cx<T> *pre) {
    const int64_t n = pb.n;
    const double *nrm = pb.p0->p.unrm.as<double>();
    const bool f32 = sizeof(T) == sizeof(float);
    cx<T> *a0 = (f32 ? pb.a0s : pb.a0).template as<cx<T>>(), *b0 = (f32 ? pb.b0s : pb.b0).template as<cx<T>>(),
          *y0 = (f32 ? pb.y0s : pb.y0).template as<cx<T>>();
    const cx<T> *minv = (f32 ? pb.minv32 : pb.minv).template as<cx<T>>();
    Plan &P0 = f32 ? pb.p032->p : pb.p0->p;
    cx<T> *xw = const_cast<cx<T> *>(x);
    if (!pb.adjoint) {
        k_ibc_split<T><<<gridn(n * nrhs), TPB, 0, s>>>(pre ? minv : nullptr, pre, xw, nrm, n, nrhs, pb.cibc, b0);
        FMB_LAUNCH_CHECK();
        run_matvec(P0, x, b0, y0, nrhs, s);
        k_ibc_combine<T><<<gridn(n * nrhs * 3), TPB, 0, s>>>(x, y0, n * nrhs * 3, r);
    } else {
        if (pre) {
            k_ibc_adj_precond<T><<<gridn(n * nrhs), TPB, 0, s>>>(minv, pre, xw, n, nrhs);
            FMB_LAUNCH_CHECK();
        }
        run_matvec_adjoint(P0, x, a0, b0, nrhs, s);
        k_ibc_adj_combine<T><<<gridn(n * nrhs), TPB, 0, s>>>(x, nrm, n, nrhs, pb.cibc, a0, b0, r);
    }
    FMB_LAUNCH_CHECK();
}

// A^H x; with pre = v, x is first set to M^{-H} v, fused with the split.
template <typename T>
static void bem_apply_adjoint_t(fmb_problem_s &pb, const cx<T> *x, cx<T> *r, int nrhs, hipStream_t s,
                                const cx<T> *pre) {
    if (pb.ibc) {
        const bool was = pb.adjoint;
        pb.adjoint = true;
        ibc_apply_t<T>(pb, x, r, nrhs, s, pre);
        pb.adjoint = was;
        return;
    }
    const int64_t n = pb.n;
    const Regions R = regions_of(pb);
    const double *nrm = pb.p0->p.unrm.as<double>();
    const bool f32 = sizeof(T) == sizeof(float);
    cx<T> *a0 = (f32 ? pb.a0s : pb.a0).template as<cx<T>>(), *b0 = (f32 ? pb.b0s : pb.b0).template as<cx<T>>(),
          *a1 = (f32 ? pb.a1s : pb.a1).template as<cx<T>>(), *b1 = (f32 ? pb.b1s : pb.b1).template as<cx<T>>(),
          *y0 = (f32 ? pb.y0s : pb.y0).template as<cx<T>>(), *y1 = (f32 ? pb.y1s : pb.y1).template as<cx<T>>();
    if (pre) {
        k_adj_precond_split<T><<<gridn(n * nrhs), TPB, 0, s>>>((f32 ? pb.minv32 : pb.minv).template as<cx<T>>(),
                                                                pre, const_cast<cx<T> *>(x), n, nrhs, R, y0, y1);
    } else {
        k_adj_split<T><<<gridn(n * nrhs), TPB, 0, s>>>(x, n, nrhs, R, y0, y1);
    }
    FMB_LAUNCH_CHECK();
    if (pb.J == 1) {
        Plan &P0 = f32 ? pb.p032->p : pb.p0->p, &P1 = f32 ? pb.p132->p : pb.p1->p;
        adjoint_pair(pb, P0, P1, y0, a0, b0, y1, a1, b1, nrhs, s);
    } else {
        multi_products<T>(pb, true, y0, a0, b0, y1, a1, b1, nrhs, s);
    }
    k_adj_combine<T><<<gridn(n * nrhs), TPB, 0, s>>>(x, nrm, n, nrhs, R, a0, b0, a1, b1, r);
    FMB_LAUNCH_CHECK();
}

// A x with the FP64 plans (T = double) or the FP32 plans (T = float).  With
// pre = v, x is first set to M^{-1} v (the preconditioned direction), fused
// with the split.  A problem in adjoint mode applies A^H and M^{-H} instead.
template <typename T>
static void bem_apply_t(fmb_problem_s &pb, const cx<T> *x, cx<T> *r, int nrhs, hipStream_t s,
                        const cx<T> *pre = nullptr) {
    if (pb.ibc) {
        ibc_apply_t<T>(pb, x, r, nrhs, s, pre);
        return;
    }
    if (pb.adjoint) {
        bem_apply_adjoint_t<T>(pb, x, r, nrhs, s, pre);
        return;
    }
    const int64_t n = pb.n;
    const Regions R = regions_of(pb);
    const double *nrm = pb.p0->p.unrm.as<double>();
    const bool f32 = sizeof(T) == sizeof(float);
    cx<T> *a0 = (f32 ? pb.a0s : pb.a0).template as<cx<T>>(), *b0 = (f32 ? pb.b0s : pb.b0).template as<cx<T>>(),
          *a1 = (f32 ? pb.a1s : pb.a1).template as<cx<T>>(), *b1 = (f32 ? pb.b1s : pb.b1).template as<cx<T>>(),
          *y0 = (f32 ? pb.y0s : pb.y0).template as<cx<T>>(), *y1 = (f32 ? pb.y1s : pb.y1).template as<cx<T>>();
    if (pre) {
        k_precond_split<T><<<gridn(n * nrhs), TPB, 0, s>>>((f32 ? pb.minv32 : pb.minv).template as<cx<T>>(), pre,
                                                            const_cast<cx<T> *>(x), nrm, n, nrhs, R, a0, b0, a1, b1);
    } else {
        k_bem_split<T><<<gridn(n * nrhs), TPB, 0, s>>>(x, nrm, n, nrhs, R, a0, b0, a1, b1);
    }
    FMB_LAUNCH_CHECK();
    if (pb.J == 1) {
        const Plan *P0 = f32 ? &pb.p032->p : &pb.p0->p, *P1 = f32 ? &pb.p132->p : &pb.p1->p;
        fmm_pair<T>(pb, P0, P1, a0, b0, y0, a1, b1, y1, nrhs, s);
    } else {
        multi_products<T>(pb, false, a0, b0, y0, a1, b1, y1, nrhs, s);
    }
    k_bem_combine<T><<<gridn(n * nrhs), TPB, 0, s>>>(x, nrm, n, nrhs, R, y0, y1, r);
    FMB_LAUNCH_CHECK();
}

template <typename T>
static void precond_t(fmb_problem_s &pb, const cx<T> *v, cx<T> *z, int nrhs, hipStream_t s) {
    const bool f32 = sizeof(T) == sizeof(float);
    if (pb.ibc) {
        // z = M^{-1} v through the split kernel (its b output lands in the staging buffer)
        k_ibc_split<T><<<gridn(pb.n * nrhs), TPB, 0, s>>>((f32 ? pb.minv32 : pb.minv).template as<cx<T>>(), v, z,
                                                           pb.p0->p.unrm.as<double>(), pb.n, nrhs, pb.cibc,
                                                           (f32 ? pb.b0s : pb.b0).template as<cx<T>>());
        FMB_LAUNCH_CHECK();
        return;
    }
    k_precond_apply<T><<<gridn(pb.n * nrhs), TPB, 0, s>>>((f32 ? pb.minv32 : pb.minv).template as<cx<T>>(), v, z,
                                                           pb.n, nrhs);
    FMB_LAUNCH_CHECK();
}

// The preconditioner in the paper's form (Sec. 3.1): z ~ M^{-1} v (M^{-H} v in
// adjoint mode) by an inner GMRES on the block-diagonal M = A_self, at most
// PG_MAXIT steps, each right-hand side stopping at the first step whose residual
// estimate is at most PG_TOL |v|.  Classical Gram-Schmidt applied twice; the small
// least-squares problems (Givens rotations, back substitution) are solved on the
// host, with one synchronisation per step.  fGMRES keeps every z, so the inexact
// inner solve is allowed to change from step to step.
constexpr int PG_MAXIT = 10;
constexpr double PG_TOL = 1e-2;

// M (and its FP32 copy when the problem has FP32 plans), from the stored inverses
static void ensure_forward_blocks(fmb_problem_s &pb, hipStream_t s) {
    if (pb.mfwd.p) return;
    const int nb = pb.nu;
    const int64_t cnt = pb.n * nb * nb;
    pb.mfwd.alloc((size_t)cnt * sizeof(cx<double>));
    DevBuf bad;
    bad.alloc(sizeof(int32_t));
    FMB_CHECK_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    if (nb == 6)
        k_block_invert<6><<<gridn(pb.n), TPB, 0, s>>>(pb.minv.as<cx<double>>(), pb.mfwd.as<cx<double>>(), pb.n,
                                                      bad.as<int32_t>());
    else
        k_block_invert<3><<<gridn(pb.n), TPB, 0, s>>>(pb.minv.as<cx<double>>(), pb.mfwd.as<cx<double>>(), pb.n,
                                                      bad.as<int32_t>());
    FMB_LAUNCH_CHECK();
    if (pb.minv32.p) {
        pb.mfwd32.alloc((size_t)cnt * sizeof(cx<float>));
        k_to32<<<gridn(cnt), TPB, 0, s>>>(pb.mfwd.as<cx<double>>(), pb.mfwd32.as<cx<float>>(), cnt);
        FMB_LAUNCH_CHECK();
    }
    int32_t hb = 0;
    FMB_CHECK_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FMB_CHECK_HIP(hipStreamSynchronize(s));
    if (hb) {
        pb.mfwd.release();
        pb.mfwd32.release();
        throw Status{FMB_EINVAL, "a preconditioner block is singular"};
    }
}

template <typename T>
static Krylov<T> &pg_workspace(fmb_problem_s &pb) {
    std::shared_ptr<void> &slot = sizeof(T) == sizeof(float) ? pb.pg32 : pb.pg64;
    if (!slot) slot = std::shared_ptr<void>(new Krylov<T>(), [](void *p) { delete static_cast<Krylov<T> *>(p); });
    return *static_cast<Krylov<T> *>(slot.get());
}

template <typename T>
static void precond_gmres(fmb_problem_s &pb, const cx<T> *v, cx<T> *z, int nrhs, hipStream_t s) {
    const bool f32 = sizeof(T) == sizeof(float);
    const int nb = pb.nu, m = PG_MAXIT;
    const int64_t len = pb.n * nb, tot = len * nrhs;
    const cx<T> *blk = (f32 ? pb.mfwd32 : pb.mfwd).template as<cx<T>>();
    FMB_REQUIRE(blk != nullptr, "the inner-GMRES preconditioner's blocks were not built");
    Krylov<T> &K = pg_workspace<T>(pb);
    krylov_alloc(K, len, nrhs, m);
    cx<T> *U = K.V.template as<cx<T>>(), *W = K.W.template as<cx<T>>();
    int32_t *act = K.act.template as<int32_t>();
    double *hn = K.hn.template as<double>(), *hninv = K.hninv.template as<double>();
    cx<double> *h = K.h.template as<cx<double>>(), *h2 = K.h2.template as<cx<double>>();
    std::vector<int32_t> on(nrhs, 1);
    FMB_CHECK_HIP(hipMemcpyAsync(act, on.data(), nrhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
    norms(K, v, hn, hninv, s);
    k_scale_into<T><<<gridn(tot), TPB, 0, s>>>(v, hninv, U, len, nrhs, act);
    FMB_LAUNCH_CHECK();
    std::vector<double> beta(nrhs), hnh(nrhs), cs((size_t)nrhs * m, 1.0);
    std::vector<cx<double>> sn((size_t)nrhs * m, mk(0.0, 0.0)), Rm((size_t)nrhs * m * m, mk(0.0, 0.0)),
        g((size_t)nrhs * (m + 1), mk(0.0, 0.0)), hh((size_t)(m + 1) * nrhs), hh2((size_t)(m + 1) * nrhs);
    std::vector<int> kr(nrhs, -1);
    FMB_CHECK_HIP(hipMemcpyAsync(beta.data(), hn, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    FMB_CHECK_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < nrhs; ++r) {
        g[(size_t)r * (m + 1)] = mk(beta[r], 0.0);
        if (!(beta[r] > 0.0)) kr[r] = 0;
    }
    int steps = 0;
    for (int j = 0; j < m; ++j) {
        bool all = true;
        for (int r = 0; r < nrhs; ++r) all = all && kr[r] >= 0;
        if (all) break;
        k_block_mul<T><<<gridn(pb.n * nrhs), TPB, 0, s>>>(blk, nb, pb.adjoint ? 1 : 0, U + (int64_t)j * tot, W, pb.n,
                                                          nrhs);
        FMB_LAUNCH_CHECK();
        dots(K, (const cx<T> *)U, j + 1, (const cx<T> *)nullptr, (const cx<T> *)W, (const int32_t *)nullptr, h, s);
        combine(K, (const cx<T> *)U, j + 1, h, -1.0, W, act, (const int32_t *)nullptr, (double *)nullptr, s);
        dots(K, (const cx<T> *)U, j + 1, (const cx<T> *)nullptr, (const cx<T> *)W, (const int32_t *)nullptr, h2, s);
        combine(K, (const cx<T> *)U, j + 1, h2, -1.0, W, act, (const int32_t *)nullptr, (double *)nullptr, s);
        norms(K, W, hn, hninv, s);
        k_scale_into<T><<<gridn(tot), TPB, 0, s>>>(W, hninv, U + (int64_t)(j + 1) * tot, len, nrhs, act);
        FMB_LAUNCH_CHECK();
        const size_t cnt = (size_t)(j + 1) * nrhs;
        FMB_CHECK_HIP(hipMemcpyAsync(hh.data(), h, cnt * sizeof(cx<double>), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipMemcpyAsync(hh2.data(), h2, cnt * sizeof(cx<double>), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipMemcpyAsync(hnh.data(), hn, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
        steps = j + 1;
        for (int r = 0; r < nrhs; ++r) {
            if (kr[r] >= 0) continue;
            std::vector<cx<double>> col(j + 2);
            for (int i = 0; i <= j; ++i) col[i] = hh[(size_t)i * nrhs + r] + hh2[(size_t)i * nrhs + r];
            col[j + 1] = mk(hnh[r], 0.0);
            double *c = &cs[(size_t)r * m];
            cx<double> *sv = &sn[(size_t)r * m], *gr = &g[(size_t)r * (m + 1)];
            for (int i = 0; i < j; ++i) {
                const cx<double> t = c[i] * col[i] + sv[i] * col[i + 1];
                col[i + 1] = c[i] * col[i + 1] - conj(sv[i]) * col[i];
                col[i] = t;
            }
            // rotation zeroing col[j + 1]: c = |a| / rho, s = (a / |a|) conj(b) / rho
            const cx<double> a = col[j], b = col[j + 1];
            const double aa = std::sqrt(abs2(a)), rho = std::sqrt(abs2(a) + abs2(b));
            if (rho == 0.0) {
                c[j] = 1.0;
                sv[j] = mk(0.0, 0.0);
            } else if (aa == 0.0) {
                c[j] = 0.0;
                sv[j] = mk(1.0, 0.0);
            } else {
                c[j] = aa / rho;
                sv[j] = (1.0 / (aa * rho)) * (a * conj(b));
            }
            col[j] = c[j] * a + sv[j] * b;
            gr[j + 1] = -(conj(sv[j]) * gr[j]);
            gr[j] = c[j] * gr[j];
            for (int i = 0; i <= j; ++i) Rm[((size_t)r * m + i) * m + j] = col[i];
            if (std::sqrt(abs2(gr[j + 1])) <= PG_TOL * beta[r]) kr[r] = j + 1;
        }
    }
    // y from R y = g per rhs (steps taken: kr, or all steps), z = U y
    std::vector<cx<double>> y((size_t)(m + 1) * nrhs, mk(0.0, 0.0));
    for (int r = 0; r < nrhs; ++r) {
        const int k = kr[r] >= 0 ? kr[r] : steps;
        std::vector<cx<double>> yr(k, mk(0.0, 0.0));
        for (int i = k - 1; i >= 0; --i) {
            cx<double> t = g[(size_t)r * (m + 1) + i];
            for (int q = i + 1; q < k; ++q) t -= Rm[((size_t)r * m + i) * m + q] * yr[q];
            const cx<double> d = Rm[((size_t)r * m + i) * m + i];
            yr[i] = abs2(d) > 0.0 ? cdiv(t, d) : mk(0.0, 0.0);
        }
        for (int i = 0; i < k; ++i) y[(size_t)i * nrhs + r] = yr[i];
    }
    cx<double> *yd = K.y.template as<cx<double>>();
    FMB_CHECK_HIP(hipMemcpyAsync(yd, y.data(), y.size() * sizeof(cx<double>), hipMemcpyHostToDevice, s));
    FMB_CHECK_HIP(hipMemsetAsync(z, 0, tot * sizeof(cx<T>), s));
    combine(K, (const cx<T> *)U, std::max(steps, 1), yd, 1.0, z, act, (const int32_t *)nullptr, (double *)nullptr, s);
    // the host vectors above are read by the copies before the stream is left
    FMB_CHECK_HIP(hipStreamSynchronize(s));
}

// One right-preconditioned fGMRES solve of A x = b, x updated in place, with
// the FP64 operator (T = double) or the FP32 one (T = float).  Returns the
// iteration count; relres receives |b - A x| / |b| per rhs (computed with the
// operator the solve used).
// Nested mode: the preconditioner of an FP64 fGMRES is one cycle of FP32 fGMRES
// (block-preconditioned when precond is set) on A32 z = v_j, to a relative
// tolerance; flexible GMRES keeps every z_j, so the inexact inner solves enter
// the FP64 minimisation and need not contract on their own.
struct InnerSolve {
    Krylov<float> *K;
    cx<float> *r32, *d32;
    double tol;
    int maxit;
    bool reorth;
    int its;
    int *matvecs;
};

template <typename T>
static int fgmres(fmb_problem_s &pb, Krylov<T> &K, const cx<T> *b, cx<T> *x, bool x_nonzero, double tol, int maxit,
                  int precond, bool reorth, std::vector<double> &relres, std::vector<double> *hist, int &matvecs,
                  hipStream_t s, InnerSolve *inner = nullptr) {
    const int nrhs = K.nrhs, m = K.m;
    const int64_t len = K.len, tot = len * nrhs;
    cx<T> *V = K.V.template as<cx<T>>(), *Z = K.Z.template as<cx<T>>(), *W = K.W.template as<cx<T>>();
    cx<T> *R = K.r.template as<cx<T>>(), *AX = K.ax.template as<cx<T>>();
    int32_t *need = K.need.template as<int32_t>(), *actd = K.act.template as<int32_t>();
    cx<double> *h = K.h.template as<cx<double>>(), *h2 = K.h2.template as<cx<double>>();
    std::vector<double> bn(nrhs), beta(nrhs);
    std::vector<int32_t> act(nrhs), jr(nrhs);
    norms(K, b, K.bnd.template as<double>(), nullptr, s);
    FMB_CHECK_HIP(hipMemcpyAsync(bn.data(), K.bnd.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    // step results, slot j & 1: res at [slot * nrhs], brk after the 2 nrhs doubles
    double *hres = static_cast<double *>(K.step.h);
    int32_t *hbrk = reinterpret_cast<int32_t *>(hres + 2 * nrhs);
    double *dres = static_cast<double *>(K.step.d);
    int32_t *dbrk = reinterpret_cast<int32_t *>(dres + 2 * nrhs);
    if (x_nonzero) {
        bem_apply_t<T>(pb, x, AX, nrhs, s);
        ++matvecs;
        k_sub<T><<<gridn(tot), TPB, 0, s>>>(b, AX, R, tot);
        FMB_LAUNCH_CHECK();
    } else {
        FMB_CHECK_HIP(hipMemsetAsync(x, 0, tot * sizeof(cx<T>), s));
        FMB_CHECK_HIP(hipMemcpyAsync(R, b, tot * sizeof(cx<T>), hipMemcpyDeviceToDevice, s));
    }
    int its = 0;
    // iterations spent: this solve's steps plus, in nested mode, the inner steps
    // (maxit caps the total; the cap is checked between outer steps)
    auto spent = [&]() { return its + (inner ? inner->its : 0); };
    relres.assign(nrhs, 0.0);
    while (true) {
        norms(K, R, K.hn.template as<double>(), K.hninv.template as<double>(), s);
        FMB_CHECK_HIP(hipMemcpyAsync(beta.data(), K.hn.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
        bool any = false;
        for (int r = 0; r < nrhs; ++r) {
            if (!std::isfinite(beta[r])) throw Status{FMB_ENONFINITE, "non-finite residual in fGMRES"};
            relres[r] = bn[r] > 0 ? beta[r] / bn[r] : 0.0;
            act[r] = (beta[r] > tol * bn[r]) ? 1 : 0;
            any = any || act[r];
        }
        if (!any || spent() >= maxit) break;
        FMB_CHECK_HIP(hipMemcpyAsync(actd, act.data(), nrhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
        k_scale_into<T><<<gridn(tot), TPB, 0, s>>>(R, K.hninv.template as<double>(), V, len, nrhs, actd);
        FMB_LAUNCH_CHECK();
        {
            std::vector<cx<double>> g0((size_t)nrhs * (m + 1), mk(0.0, 0.0));
            for (int r = 0; r < nrhs; ++r) g0[(size_t)r * (m + 1)] = mk(beta[r], 0.0);
            FMB_CHECK_HIP(hipMemcpyAsync(K.g.p, g0.data(), g0.size() * sizeof(cx<double>), hipMemcpyHostToDevice, s));
        }
        for (int r = 0; r < nrhs; ++r) jr[r] = 0;
        // One Arnoldi step: apply, orthogonalise, rotate.  The device retires
        // converged rhs itself, so step j + 1 is enqueued before the host reads
        // step j's result: the GPU does not wait on the host between steps.
        // After the last step of a solve one masked step may have run.
        auto enqueue = [&](int j) {
            cx<T> *vj = V + (int64_t)j * tot, *zj = Z + (int64_t)j * tot;
            if constexpr (std::is_same<T, double>::value) {
                if (inner) {
                    k_to32_active<<<gridn(tot), TPB, 0, s>>>(vj, inner->r32, len, nrhs, actd);
                    FMB_LAUNCH_CHECK();
                    std::vector<double> rel;
                    inner->its += fgmres<float>(pb, *inner->K, inner->r32, inner->d32, false, inner->tol, inner->maxit,
                                                precond, inner->reorth, rel, nullptr, *inner->matvecs, s);
                    k_to64<<<gridn(tot), TPB, 0, s>>>(inner->d32, zj, tot);
                    FMB_LAUNCH_CHECK();
                    bem_apply_t<T>(pb, zj, W, nrhs, s);
                }
            }
            if (inner) {
            } else if (precond == 2) {
                precond_gmres<T>(pb, vj, zj, nrhs, s);       // z_j ~ M^{-1} v_j by the inner GMRES
                bem_apply_t<T>(pb, zj, W, nrhs, s);
            } else if (precond) {
                bem_apply_t<T>(pb, zj, W, nrhs, s, vj);      // z_j = M^{-1} v_j fused with the split
            } else {
                FMB_CHECK_HIP(hipMemcpyAsync(zj, vj, tot * sizeof(cx<T>), hipMemcpyDeviceToDevice, s));
                bem_apply_t<T>(pb, zj, W, nrhs, s);
            }
            ++matvecs;
            // classical Gram-Schmidt; the same pass yields |A z|^2 as h[j+1], the
            // update yields |W'|^2
            double *npart = K.npart.template as<double>(), *hn = K.hn.template as<double>(),
                   *hninv = K.hninv.template as<double>();
            dots(K, (const cx<T> *)V, j + 1, (const cx<T> *)W, (const cx<T> *)W, (const int32_t *)nullptr, h, s);
            combine(K, (const cx<T> *)V, j + 1, h, -1.0, W, actd, (const int32_t *)nullptr, npart, s);
            k_post1<<<nrhs, 64, 0, s>>>(npart, K.nchc, h, j, actd, need, hn, hninv, nrhs);
            FMB_LAUNCH_CHECK();
            // second pass only where the DGKS test asks for it (solves with reorth)
            if (reorth) {
                dots(K, (const cx<T> *)V, j + 1, (const cx<T> *)nullptr, (const cx<T> *)W, (const int32_t *)need, h2,
                     s);
                combine(K, (const cx<T> *)V, j + 1, h2, -1.0, W, actd, (const int32_t *)need, (double *)nullptr, s);
                k_post2<<<nrhs, 64, 0, s>>>(h, h2, j + 1, need, hn, hninv, nrhs);
            }
            k_scale_into<T><<<gridn(tot), TPB, 0, s>>>(W, hninv, V + (int64_t)(j + 1) * tot, len, nrhs, actd);
            const int sl = j & 1;
            k_givens<<<nrhs, 64, (size_t)(2 * j + 2) * sizeof(cx<double>) + (size_t)j * sizeof(double), s>>>(
                K.H.template as<cx<double>>(), m + 1, j, h, hn, K.cs.template as<double>(),
                K.sn.template as<cx<double>>(), K.g.template as<cx<double>>(), actd, K.bnd.template as<double>(), tol,
                dres + sl * nrhs, dbrk + sl * nrhs, nrhs, m);
            FMB_LAUNCH_CHECK();
            FMB_CHECK_HIP(hipEventRecord(K.ev[sl], s));
        };
        int queued = -1;
        for (int j = 0; j < m && spent() < maxit; ++j) {
            if (queued < j) {
                enqueue(j);
                queued = j;
            }
            if (j + 1 < m && spent() + 1 < maxit) {
                enqueue(j + 1);
                queued = j + 1;
            }
            const int sl = j & 1;
            FMB_CHECK_HIP(hipEventSynchronize(K.ev[sl]));
            ++its;
            bool more = false;
            double worst = 0.0;
            for (int r = 0; r < nrhs; ++r) {
                if (!act[r]) continue;
                jr[r] = j + 1;
                const double rs = hres[sl * nrhs + r];
                if (!std::isfinite(rs)) throw Status{FMB_ENONFINITE, "non-finite Arnoldi step in fGMRES"};
                worst = std::max(worst, bn[r] > 0 ? rs / bn[r] : 0.0);
                if (rs <= tol * bn[r] || hbrk[sl * nrhs + r]) {
                    act[r] = 0;                       // retired on the device by the same rule
                } else {
                    more = true;
                }
            }
            if (hist) hist->push_back(worst);
            if (!more) break;
        }
        // x += Z y with y = H^{-1} g per rhs
        FMB_CHECK_HIP(hipMemcpyAsync(K.jr.p, jr.data(), nrhs * sizeof(int32_t), hipMemcpyHostToDevice, s));
        k_trisolve<<<1, 1024, 0, s>>>(K.H.template as<cx<double>>(), m + 1, K.g.template as<cx<double>>(),
                                      K.jr.template as<int32_t>(), K.y.template as<cx<double>>(), nrhs, m);
        int jmax = 0;
        for (int r = 0; r < nrhs; ++r) jmax = std::max(jmax, jr[r]);
        if (jmax > 0)
            combine(K, (const cx<T> *)Z, jmax, (const cx<double> *)K.y.template as<cx<double>>(), 1.0, x,
                    (const int32_t *)nullptr, (const int32_t *)nullptr, (double *)nullptr, s);
        FMB_LAUNCH_CHECK();
        // true residual
        bem_apply_t<T>(pb, x, AX, nrhs, s);
        ++matvecs;
        k_sub<T><<<gridn(tot), TPB, 0, s>>>(b, AX, R, tot);
        FMB_LAUNCH_CHECK();
    }
    return its;
}

static fmb_gmres_opts solve_opts(const fmb_gmres_opts *o) {
    fmb_gmres_opts op;
    fmb_gmres_opts_default(&op);
    if (o) op = *o;
    return op;
}

static void check_solve_args(fmb_problem_s *pb, const void *rhs, const void *x, int nrhs, const fmb_gmres_opts &op) {
    FMB_REQUIRE(pb && rhs && x && rhs != x, "bad arguments");
    FMB_REQUIRE(nrhs >= 1 && nrhs <= pb->nrhs_max, "nrhs out of range");
    FMB_REQUIRE(op.tol > 0 && op.restart >= 1 && op.maxit >= 1, "bad solver options");
    FMB_REQUIRE(op.mixed >= 0 && op.mixed <= 2, "mixed must be 0, 1 or 2");
    FMB_REQUIRE(op.precond >= 0 && op.precond <= 2, "precond must be 0, 1 or 2");
    FMB_REQUIRE(!op.mixed || pb->p032, "mixed precision needs the FP32 plans");
}

// FP64 fGMRES on the FP64 plans (basis op.restart), each step preconditioned by
// one FP32 fGMRES cycle of at most `inner` steps to op.inner_tol; returns the
// outer steps and adds outer plus inner steps to its.
static int nested_fgmres(fmb_problem_s *pb, Krylov<double> &K, Krylov<float> &K32, cx<float> *r32, cx<float> *d32,
                         const cx<double> *b, cx<double> *X, int nrhs, bool x0, int inner, int maxit,
                         const fmb_gmres_opts &op, std::vector<double> &relres, std::vector<double> &hist, int &its,
                         int &mv64, int &mv32, hipStream_t s) {
    const int64_t len = pb->n * pb->nu;
    const int mi = std::max(1, inner);
    krylov_alloc(K, len, nrhs, op.restart);
    krylov_alloc(K32, len, nrhs, mi);
    InnerSolve in{&K32, r32, d32, op.inner_tol, mi, op.inner_reorth != 0, 0, &mv32};
    const int outer = fgmres<double>(*pb, K, b, X, x0, op.tol, maxit, op.precond, true, relres, &hist, mv64, s, &in);
    its += outer + in.its;
    return outer;
}

// One complete solve on stream s; returns whether the tolerance was reached.
static bool solve_one(fmb_problem_s *pb, const void *rhs, void *x, int32_t nrhs, const fmb_gmres_opts &op,
                      fmb_gmres_info *info, hipStream_t s) {
    check_solve_args(pb, rhs, x, nrhs, op);
    if (op.precond == 2) ensure_forward_blocks(*pb, s);
    pb->serial = op.serial != 0;
    pb->adjoint = op.adjoint != 0;
    struct ModeReset {
        fmb_problem_s *p;
        ~ModeReset() {
            p->serial = false;
            p->adjoint = false;
        }
    } mode_reset{pb};
    const int64_t len = pb->n * pb->nu, tot = len * nrhs;
    const cx<double> *b = (const cx<double> *)rhs;
    cx<double> *X = (cx<double> *)x;
    std::vector<double> relres, hist;
    int mv64 = 0, mv32 = 0, its = 0, refinements = 0;
    bool fallback = false;
    double final_res = 0.0;
    Krylov<double> K;
    if (!op.mixed) {
        krylov_alloc(K, len, nrhs, op.restart);
        its = fgmres<double>(*pb, K, b, X, op.x0_given != 0, op.tol, op.maxit, op.precond, true, relres, &hist, mv64,
                             s);
        for (double v : relres) final_res = std::max(final_res, v);
    } else if (op.mixed == 2) {
        // nested: FP64 fGMRES whose preconditioner is one FP32 fGMRES cycle
        Krylov<float> K32;
        DevBuf r32, d32;
        r32.alloc(tot * sizeof(cx<float>));
        d32.alloc(tot * sizeof(cx<float>));
        refinements = nested_fgmres(pb, K, K32, r32.as<cx<float>>(), d32.as<cx<float>>(), b, X, nrhs,
                                    op.x0_given != 0, std::min(op.restart, op.inner_maxit), op.maxit, op, relres, hist,
                                    its, mv64, mv32, s);
        for (double v : relres) final_res = std::max(final_res, v);
    } else {
        // iterative refinement: FP64 residuals r = b - A64 x, inner fGMRES on
        // A32 d = r with FP32 Krylov vectors, x += d
        krylov_alloc(K, len, nrhs, 1);                  // FP64 norms only
        Krylov<float> K32;
        krylov_alloc(K32, len, nrhs, op.restart);
        DevBuf rr, ax, r32, d32;
        rr.alloc(tot * sizeof(cx<double>));
        ax.alloc(tot * sizeof(cx<double>));
        r32.alloc(tot * sizeof(cx<float>));
        d32.alloc(tot * sizeof(cx<float>));
        if (op.x0_given) {
            bem_apply_t<double>(*pb, X, ax.as<cx<double>>(), nrhs, s);
            ++mv64;
            k_sub<double><<<gridn(tot), TPB, 0, s>>>(b, ax.as<cx<double>>(), rr.as<cx<double>>(), tot);
        } else {
            FMB_CHECK_HIP(hipMemsetAsync(X, 0, tot * sizeof(cx<double>), s));
            FMB_CHECK_HIP(hipMemcpyAsync(rr.p, b, tot * sizeof(cx<double>), hipMemcpyDeviceToDevice, s));
        }
        std::vector<double> bn(nrhs), rn(nrhs);
        double prev_res = 0.0, prev_itol = 0.5;
        norms(K, b, K.hn.as<double>(), nullptr, s);
        FMB_CHECK_HIP(hipMemcpyAsync(bn.data(), K.hn.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        while (true) {
            norms(K, (const cx<double> *)rr.as<cx<double>>(), K.hn.as<double>(), nullptr, s);
            FMB_CHECK_HIP(hipMemcpyAsync(rn.data(), K.hn.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
            FMB_CHECK_HIP(hipStreamSynchronize(s));
            final_res = 0.0;
            for (int r = 0; r < nrhs; ++r) {
                if (!std::isfinite(rn[r])) throw Status{FMB_ENONFINITE, "non-finite residual in refinement"};
                final_res = std::max(final_res, bn[r] > 0 ? rn[r] / bn[r] : 0.0);
            }
            hist.push_back(final_res);
            if (final_res <= op.tol || its >= op.maxit || refinements >= 50) break;
            // a step that cut the residual by less than 2x, or by less than 1/20 of what its inner
            // tolerance asked for: the FP32 operator (or its inner solve) no longer contracts the FP64
            // residual, so go on in nested mode from the current iterate
            if (refinements >= 1 && final_res > std::min(0.5, 20.0 * prev_itol) * prev_res) {
                fallback = true;
                break;
            }
            prev_res = final_res;
            std::vector<double> inner;
            // the last refinements only need to close the gap to tol: loosen the inner tolerance to
            // a fraction of tol/|r| when that is looser than the configured one
            const double itol = std::min(0.5, std::max(op.inner_tol, 0.3 * op.tol / std::max(final_res, 1e-300)));
            prev_itol = itol;
            k_to32<<<gridn(tot), TPB, 0, s>>>(rr.as<cx<double>>(), r32.as<cx<float>>(), tot);
            FMB_LAUNCH_CHECK();
            its += fgmres<float>(*pb, K32, r32.as<cx<float>>(), d32.as<cx<float>>(), false, itol,
                                 std::min(op.inner_maxit, op.maxit - its), op.precond, op.inner_reorth != 0, inner, nullptr, mv32, s);
            k_add_from32<<<gridn(tot), TPB, 0, s>>>(X, d32.as<cx<float>>(), tot);
            bem_apply_t<double>(*pb, X, ax.as<cx<double>>(), nrhs, s);
            ++mv64;
            k_sub<double><<<gridn(tot), TPB, 0, s>>>(b, ax.as<cx<double>>(), rr.as<cx<double>>(), tot);
            FMB_LAUNCH_CHECK();
            ++refinements;
        }
        if (fallback) {
            // go on from X in nested mode, with inner cycles of at most 100 steps
            std::vector<double> rel;
            nested_fgmres(pb, K, K32, r32.as<cx<float>>(), d32.as<cx<float>>(), b, X, nrhs, true,
                          std::min({op.restart, op.inner_maxit, 100}), std::max(1, op.maxit - its), op, rel, hist, its,
                          mv64, mv32, s);
            final_res = 0.0;
            for (double v : rel) final_res = std::max(final_res, v);
        }
    }
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->iterations = its;
        info->refinements = refinements;
        info->matvecs64 = mv64;
        info->matvecs32 = mv32;
        info->fp64_fallback = fallback ? 1 : 0;
        info->residual = final_res;
        for (size_t i = 0; i < hist.size() && i < 256; ++i) info->history[i] = hist[i];
    }
    return final_res <= op.tol;
}

}  // namespace fmb

using namespace fmb;

extern "C" {

int fmb_gmres_opts_default(fmb_gmres_opts *o) {
    if (!o) return FMB_EINVAL;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-6;
    o->restart = 100;
    o->maxit = 1000;
    o->precond = 1;
    o->inner_tol = 1e-3;
    o->inner_maxit = 300;
    return FMB_OK;
}

namespace fmb {

// Shared set-up of a dielectric problem with J scatterers: staging buffers,
// the 6x6 preconditioner blocks and the streams.  h->p0, pj, pj32, J, reg,
// loc, off, nj, tcj, gamj are filled in by the caller.
static void setup_dielectric(fmb_problem_s *h, hipStream_t s) {
    const Plan &A = h->p0->p;
    int nr = A.nrhs_max;
    for (int j = 0; j < h->J; ++j) {
        nr = std::min(nr, h->pj[j]->p.nrhs_max);
        if (h->p032) nr = std::min(nr, h->pj32[j]->p.nrhs_max);
    }
    if (h->p032) nr = std::min(nr, h->p032->p.nrhs_max);
    h->nrhs_max = nr;
    int64_t o = 0;
    for (int j = 0; j < h->J; ++j) {
        h->off[j] = o;
        o += (int64_t)nr * 3 * h->nj[j];
    }
    const size_t m3 = (size_t)A.n * 3 * nr;
    for (DevBuf *d : {&h->a0, &h->b0, &h->a1, &h->b1, &h->y0, &h->y1}) d->alloc(m3 * sizeof(cx<double>));
    if (h->p032)
        for (DevBuf *d : {&h->a0s, &h->b0s, &h->a1s, &h->b1s, &h->y0s, &h->y1s}) d->alloc(m3 * sizeof(cx<float>));
    h->minv.alloc((size_t)A.n * 36 * sizeof(cx<double>));
    RegionCorr C{};
    for (int j = 0; j < h->J; ++j) {
        const Plan &B = h->pj[j]->p;
        C.cv[j] = B.corr_v.as<cx<double>>();
        C.cg[j] = B.corr_g.as<cx<double>>();
        C.tri_nodes[j] = B.tri_nodes.as<int32_t>();
        C.point_tri[j] = B.point_tri.as<int32_t>();
    }
    DevBuf bad;
    bad.alloc(sizeof(int32_t));
    FMB_CHECK_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
    k_precond_build<<<gridn(A.n), TPB, 0, s>>>(A.unrm.as<double>(), A.point_tri.as<int32_t>(),
                                                A.tri_nodes.as<int32_t>(), (int)A.tri_m, A.corr_v.as<cx<double>>(),
                                                A.corr_g.as<cx<double>>(), C, regions_of(*h), A.n,
                                                h->minv.as<cx<double>>(), bad.as<int32_t>());
    FMB_LAUNCH_CHECK();
    int32_t hb = 0;
    FMB_CHECK_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    FMB_CHECK_HIP(hipStreamSynchronize(s));
    FMB_REQUIRE(hb == 0, "a 6x6 self block of the preconditioner is singular");
    if (h->p032) {
        h->minv32.alloc((size_t)A.n * 36 * sizeof(cx<float>));
        k_to32<<<gridn(A.n * 36), TPB, 0, s>>>(h->minv.as<cx<double>>(), h->minv32.as<cx<float>>(), A.n * 36);
        FMB_LAUNCH_CHECK();
        FMB_CHECK_HIP(hipStreamSynchronize(s));
    }
    FMB_CHECK_HIP(hipStreamCreateWithFlags(&h->s2, hipStreamNonBlocking));
    FMB_CHECK_HIP(hipStreamCreateWithFlags(&h->s1, hipStreamNonBlocking));
    for (hipEvent_t *e : {&h->ev_fork, &h->ev_join, &h->ev_in, &h->ev_out})
        FMB_CHECK_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
}

static void check_plans(const Plan &A, const Plan &B, const char *what) {
    FMB_REQUIRE(B.precision == A.precision, what);
    FMB_REQUIRE(B.corr_mode != FMB_CORR_NONE && B.tri_m == A.tri_m,
                "the BEM system needs self-triangle corrections in every plan");
}

}  // namespace fmb

// The interior plan of a scatterer must carry k_j = k0 sqrt(eps_j mu_j) with the
// principal square root (Im k_j >= 0 for passive media; Sec. 2.1) and an FP32 plan the wavenumber of
// its FP64 twin: a mismatched plan would silently build another system.
static void check_wavenumber(const Plan &P, cx<double> want, const char *what) {
    const cx<double> got = mk(P.k_re, P.k_im);
    FMB_REQUIRE(abs2(got - want) <= 1e-18 * std::max(abs2(want), 1e-300),
                std::string(what) + ": the plan's wavenumber does not match");
}

static cx<double> interior_k(const Plan &A, cx<double> e, cx<double> u) {
    const std::complex<double> r = std::sqrt(std::complex<double>(e.re, e.im) * std::complex<double>(u.re, u.im));
    const std::complex<double> k = std::complex<double>(A.k_re, A.k_im) * r;   // principal square root
    return mk(k.real(), k.imag());
}

int bem_problem_create(fmb_plan_t p0, fmb_plan_t p1, fmb_plan_t p0_32, fmb_plan_t p1_32, const double *eps,
                       const double *mu, void *stream, fmb_problem_t *out) {
    return guarded([&] {
        FMB_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        FMB_REQUIRE(p0 && p1, "plans p0 and p1 are required");
        FMB_REQUIRE(eps && mu, "eps and mu are required");
        const Plan &A = p0->p, &B = p1->p;
        FMB_REQUIRE(A.n == B.n, "plans cover different node counts");
        FMB_REQUIRE(A.precision == FMB_FP64 && B.precision == FMB_FP64, "p0 and p1 must be FP64 plans");
        FMB_REQUIRE(A.corr_mode != FMB_CORR_NONE, "the BEM system needs self-triangle corrections in both plans");
        check_plans(A, B, "p0 and p1 must be FP64 plans");
        FMB_REQUIRE((p0_32 == nullptr) == (p1_32 == nullptr), "give both FP32 plans or neither");
        // the two products of an application run concurrently on the plans' own workspaces
        FMB_REQUIRE(p0 != p1, "p0 and p1 must be two different plans");
        if (p0_32) {
            FMB_REQUIRE(p0_32 != p1_32, "p0_32 and p1_32 must be two different plans");
            FMB_REQUIRE(p0_32->p.n == A.n && p1_32->p.n == A.n, "FP32 plans cover different node counts");
            FMB_REQUIRE(p0_32->p.precision == FMB_FP32 && p1_32->p.precision == FMB_FP32, "p0_32/p1_32 must be FP32");
        }
        cx<double> e = mk(eps[0], eps[1]), u = mk(mu[0], mu[1]);
        FMB_REQUIRE(abs2(e) > 0.0, "eps must be non-zero");
        check_wavenumber(B, interior_k(A, e, u), "p1 (k1 = k0 sqrt(eps mu))");
        if (p0_32) {
            check_wavenumber(p0_32->p, mk(A.k_re, A.k_im), "p0_32 (k0)");
            check_wavenumber(p1_32->p, mk(B.k_re, B.k_im), "p1_32 (k1)");
        }
        auto *h = new fmb_problem_s;
        std::unique_ptr<fmb_problem_s> guard(h);
        h->p0 = p0;
        h->p1 = p1;
        h->p032 = p0_32;
        h->p132 = p1_32;
        h->n = A.n;
        h->eps = e;
        h->mu = u;
        h->gamma = u;
        h->k0_re = A.k_re;
        h->k0_im = A.k_im;
        h->J = 1;
        h->pj[0] = p1;
        h->pj32[0] = p1_32;
        h->nj[0] = A.n;
        h->tcj[0] = cdiv(mk(1.0, 0.0) - e, e);
        h->gamj[0] = u;
        setup_dielectric(h, (hipStream_t)stream);
        *out = guard.release();
    });
}

int bem_problem_create_multi(fmb_plan_t p0, const fmb_plan_t *pj, int32_t J, const int32_t *region,
                             const double *eps, const double *mu, fmb_plan_t p0_32, const fmb_plan_t *pj_32,
                             void *stream, fmb_problem_t *out) {
    return guarded([&] {
        FMB_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        FMB_REQUIRE(p0 && pj && region && eps && mu, "p0, pj, region, eps and mu are required");
        FMB_REQUIRE(J >= 1 && J <= MAXJ, "J must be in [1, 8]");
        const Plan &A = p0->p;
        FMB_REQUIRE(A.precision == FMB_FP64 && A.corr_mode != FMB_CORR_NONE,
                    "p0 must be an FP64 plan with self-triangle corrections");
        FMB_REQUIRE((p0_32 == nullptr) == (pj_32 == nullptr), "give the FP32 host plan and FP32 scatterer plans together");
        std::vector<int32_t> loc(A.n);
        std::vector<int64_t> cnt(J, 0);
        for (int64_t a = 0; a < A.n; ++a) {
            FMB_REQUIRE(region[a] >= 0 && region[a] < J, "region out of range");
            loc[a] = (int32_t)cnt[region[a]]++;
        }
        auto *h = new fmb_problem_s;
        std::unique_ptr<fmb_problem_s> guard(h);
        for (int j = 0; j < J; ++j) {
            FMB_REQUIRE(pj[j] != nullptr, "a scatterer plan is NULL");
            FMB_REQUIRE(pj[j]->p.n == cnt[j], "scatterer plan j must hold exactly the nodes with region j");
            check_plans(A, pj[j]->p, "scatterer plans must be FP64");
            FMB_REQUIRE(pj[j] != p0, "a scatterer plan must differ from p0");
            for (int i = 0; i < j; ++i) FMB_REQUIRE(pj[i] != pj[j], "scatterer plans must be different plans");
            if (p0_32) {
                FMB_REQUIRE(pj_32[j] && pj_32[j]->p.n == cnt[j] && pj_32[j]->p.precision == FMB_FP32,
                            "FP32 scatterer plan j must hold the nodes with region j");
                FMB_REQUIRE(pj_32[j] != p0_32, "an FP32 scatterer plan must differ from p0_32");
                for (int i = 0; i < j; ++i) FMB_REQUIRE(pj_32[i] != pj_32[j], "FP32 scatterer plans must be different plans");
                check_wavenumber(pj_32[j]->p, mk(pj[j]->p.k_re, pj[j]->p.k_im), "FP32 scatterer plan");
            }
            const cx<double> e = mk(eps[2 * j], eps[2 * j + 1]), u = mk(mu[2 * j], mu[2 * j + 1]);
            FMB_REQUIRE(abs2(e) > 0.0, "eps must be non-zero");
            check_wavenumber(pj[j]->p, interior_k(A, e, u), "scatterer plan (k_j = k0 sqrt(eps_j mu_j))");
            h->pj[j] = pj[j];
            h->pj32[j] = p0_32 ? pj_32[j] : nullptr;
            h->nj[j] = cnt[j];
            h->tcj[j] = cdiv(mk(1.0, 0.0) - e, e);
            h->gamj[j] = u;
        }
        if (p0_32) {
            FMB_REQUIRE(p0_32->p.n == A.n && p0_32->p.precision == FMB_FP32, "p0_32 must be an FP32 host plan");
            check_wavenumber(p0_32->p, mk(A.k_re, A.k_im), "p0_32 (k0)");
        }
        h->p0 = p0;
        h->p1 = pj[0];
        h->p032 = p0_32;
        h->p132 = p0_32 ? pj_32[0] : nullptr;
        h->n = A.n;
        h->eps = mk(eps[0], eps[1]);
        h->mu = mk(mu[0], mu[1]);
        h->gamma = h->mu;
        h->k0_re = A.k_re;
        h->k0_im = A.k_im;
        h->J = J;
        hipStream_t s = (hipStream_t)stream;
        if (J > 1) {
            h->reg.alloc((size_t)A.n * sizeof(int32_t));
            h->loc.alloc((size_t)A.n * sizeof(int32_t));
            FMB_CHECK_HIP(hipMemcpyAsync(h->reg.p, region, (size_t)A.n * sizeof(int32_t), hipMemcpyHostToDevice, s));
            FMB_CHECK_HIP(hipMemcpyAsync(h->loc.p, loc.data(), (size_t)A.n * sizeof(int32_t), hipMemcpyHostToDevice, s));
        }
        setup_dielectric(h, s);
        *out = guard.release();
    });
}

int bem_problem_create_ibc(fmb_plan_t p0, fmb_plan_t p0_32, const double *Z, void *stream, fmb_problem_t *out) {
    return guarded([&] {
        FMB_REQUIRE(out != nullptr, "out is NULL");
        *out = nullptr;
        FMB_REQUIRE(p0 != nullptr && Z != nullptr, "the k0 plan and Z are required");
        const Plan &A = p0->p;
        FMB_REQUIRE(A.precision == FMB_FP64, "p0 must be an FP64 plan");
        FMB_REQUIRE(A.corr_mode != FMB_CORR_NONE, "the IBC system needs self-triangle corrections");
        if (p0_32) {
            FMB_REQUIRE(p0_32->p.n == A.n && p0_32->p.precision == FMB_FP32, "p0_32 must be an FP32 plan of the nodes");
            FMB_REQUIRE(p0_32->p.k_re == A.k_re && p0_32->p.k_im == A.k_im, "p0_32 must have the wavenumber of p0");
        }
        const cx<double> z = mk(Z[0], Z[1]);
        FMB_REQUIRE(std::isfinite(z.re) && std::isfinite(z.im) && abs2(z) > 0.0, "Z must be finite and non-zero");
        hipStream_t s = (hipStream_t)stream;
        auto *h = new fmb_problem_s;
        std::unique_ptr<fmb_problem_s> guard(h);
        h->p0 = p0;
        h->p032 = p0_32;
        h->ibc = true;
        h->nu = 3;
        h->n = A.n;
        h->eps = mk(1.0, 0.0);
        h->mu = mk(1.0, 0.0);
        h->gamma = h->mu;
        h->k0_re = A.k_re;
        h->k0_im = A.k_im;
        h->cibc = cdiv(mk(-A.k_im, A.k_re), z);              // i k0 / Z
        int nr = A.nrhs_max;
        if (p0_32) nr = std::min(nr, p0_32->p.nrhs_max);
        h->nrhs_max = nr;
        const size_t m3 = (size_t)A.n * 3 * nr;
        for (DevBuf *d : {&h->a0, &h->b0, &h->y0}) d->alloc(m3 * sizeof(cx<double>));
        if (p0_32)
            for (DevBuf *d : {&h->a0s, &h->b0s, &h->y0s}) d->alloc(m3 * sizeof(cx<float>));
        h->minv.alloc((size_t)A.n * 9 * sizeof(cx<double>));
        DevBuf bad;
        bad.alloc(sizeof(int32_t));
        FMB_CHECK_HIP(hipMemsetAsync(bad.p, 0, sizeof(int32_t), s));
        k_ibc_precond_build<<<gridn(A.n), TPB, 0, s>>>(A.unrm.as<double>(), A.point_tri.as<int32_t>(),
                                                        A.tri_nodes.as<int32_t>(), (int)A.tri_m,
                                                        A.corr_v.as<cx<double>>(), A.corr_g.as<cx<double>>(), A.n,
                                                        h->cibc, h->minv.as<cx<double>>(), bad.as<int32_t>());
        FMB_LAUNCH_CHECK();
        int32_t hb = 0;
        FMB_CHECK_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
        FMB_REQUIRE(hb == 0, "a 3x3 self block of the preconditioner is singular");
        if (p0_32) {
            h->minv32.alloc((size_t)A.n * 9 * sizeof(cx<float>));
            k_to32<<<gridn(A.n * 9), TPB, 0, s>>>(h->minv.as<cx<double>>(), h->minv32.as<cx<float>>(), A.n * 9);
            FMB_LAUNCH_CHECK();
            FMB_CHECK_HIP(hipStreamSynchronize(s));
        }
        FMB_CHECK_HIP(hipStreamCreateWithFlags(&h->s2, hipStreamNonBlocking));
        FMB_CHECK_HIP(hipStreamCreateWithFlags(&h->s1, hipStreamNonBlocking));
        for (hipEvent_t *e : {&h->ev_fork, &h->ev_join, &h->ev_in, &h->ev_out})
            FMB_CHECK_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
        *out = guard.release();
    });
}

}  // extern "C"

namespace {

// The field sums of bem_field and bem_field_noalloc.  `staging` is device memory
// for the nt target points, or NULL to allocate it for this call.
void field_sums(fmb_problem_t pb, const void *x, int32_t nrhs, const double *points, int64_t nt, int32_t region,
                int32_t far, void *E, hipStream_t s, double *staging) {
    FMB_REQUIRE(pb && x && points && E, "bad arguments");
    FMB_REQUIRE(nrhs >= 1 && nrhs <= pb->nrhs_max, "nrhs out of range");
    FMB_REQUIRE(nt >= 1, "no target points");
    FMB_REQUIRE(region == 0 || (region == 1 && !pb->ibc && pb->J == 1),
                "region must be 0 (host) or 1 (interior of a one-scatterer dielectric problem)");
    FMB_REQUIRE(far >= 0 && far <= 2, "kind must be 0 (field), 1 (far field) or 2 (curl)");
    FMB_REQUIRE(far == 0 || region == 0, "the far field and the curl are of the host region");
    for (int64_t i = 0; i < 3 * nt; ++i) FMB_REQUIRE(std::isfinite(points[i]), "non-finite target point");
    if (far == 1)
        for (int64_t i = 0; i < nt; ++i) {
            const double r2 = points[3 * i] * points[3 * i] + points[3 * i + 1] * points[3 * i + 1] +
                              points[3 * i + 2] * points[3 * i + 2];
            FMB_REQUIRE(std::fabs(r2 - 1.0) <= 1e-9, "far-field directions must be unit vectors");
        }
    const Plan &A = pb->p0->p;
    const Plan &K = region == 1 ? pb->p1->p : A;
    DevBuf dt;
    if (!staging) {
        dt.alloc((size_t)nt * 3 * sizeof(double));
        staging = dt.as<double>();
    }
    FMB_CHECK_HIP(hipMemcpyAsync(staging, points, (size_t)nt * 3 * sizeof(double), hipMemcpyHostToDevice, s));
    const cx<double> tc = cdiv(mk(1.0, 0.0) - pb->eps, pb->eps);
    const dim3 grid((unsigned)((nt + FE_TILE - 1) / FE_TILE), (unsigned)nrhs);
    auto kern = far == 1 ? k_field<1> : (far == 2 ? k_field<2> : k_field<0>);
    kern<<<grid, FE_TILE, 0, s>>>(staging, nt, A.spts.as<double>(), A.snrm.as<double>(), A.sw.as<double>(),
                                  A.perm.as<int32_t>(), (const cx<double> *)x, pb->n, pb->nu, region,
                                  pb->ibc ? 1 : 0, K.k_re, K.k_im, tc, pb->gamma, pb->cibc, (cx<double> *)E);
    FMB_LAUNCH_CHECK();
    FMB_CHECK_HIP(hipStreamSynchronize(s));
}

// Scratch of bem_field_noalloc: the staged target points.  Each GPU holds its
// own copy of this array from the library's load to the process's end; host
// code uses only the device address that hipGetSymbolAddress returns for it.
constexpr int64_t FIELD_NOALLOC_MAX = FMB_FIELD_NOALLOC_MAX_TARGETS;
__device__ __align__(256) double scratch[FIELD_NOALLOC_MAX * 3];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[MAX_DEVICES] = {};

// The current device's address of `scratch`, looked up on the first call on
// that device (with it current) and kept.
double *scratch_for_current_device() {
    int dev = 0;
    FMB_CHECK_HIP(hipGetDevice(&dev));
    FMB_REQUIRE(dev >= 0 && dev < MAX_DEVICES, "device index out of range for bem_field_noalloc");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        FMB_CHECK_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        FMB_REQUIRE(ptr != nullptr, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int bem_field(fmb_problem_t pb, const void *x, int32_t nrhs, const double *points, int64_t nt, int32_t region,
              int32_t far, void *E, void *stream) {
    return guarded([&] { field_sums(pb, x, nrhs, points, nt, region, far, E, (hipStream_t)stream, nullptr); });
}

int bem_field_noalloc(fmb_problem_t pb, const void *x, int32_t nrhs, const double *points, int64_t nt,
                      int32_t region, int32_t far, void *E, void *stream) {
    return guarded([&] {
        FMB_REQUIRE(nt <= FIELD_NOALLOC_MAX, "bem_field_noalloc takes at most " +
                                                 std::to_string(FIELD_NOALLOC_MAX) + " target points per call");
        double *staging = scratch_for_current_device();
        field_sums(pb, x, nrhs, points, nt, region, far, E, (hipStream_t)stream, staging);
    });
}

int bem_far_field_adjoint(fmb_problem_t pb, const void *G, int32_t nrhs, const double *dirs, int64_t nd, void *xbar,
                          void *stream) {
    return guarded([&] {
        FMB_REQUIRE(pb && G && dirs && xbar, "bad arguments");
        FMB_REQUIRE(nrhs >= 1 && nrhs <= pb->nrhs_max, "nrhs out of range");
        FMB_REQUIRE(nd >= 1, "no directions");
        for (int64_t i = 0; i < nd; ++i) {
            const double r2 = dirs[3 * i] * dirs[3 * i] + dirs[3 * i + 1] * dirs[3 * i + 1] + dirs[3 * i + 2] * dirs[3 * i + 2];
            FMB_REQUIRE(std::isfinite(r2) && std::fabs(r2 - 1.0) <= 1e-9, "directions must be unit vectors");
        }
        hipStream_t s = (hipStream_t)stream;
        const Plan &A = pb->p0->p;
        DevBuf dd;
        dd.alloc((size_t)nd * 3 * sizeof(double));
        FMB_CHECK_HIP(hipMemcpyAsync(dd.p, dirs, (size_t)nd * 3 * sizeof(double), hipMemcpyHostToDevice, s));
        const dim3 grid((unsigned)((pb->n + FE_TILE - 1) / FE_TILE), (unsigned)nrhs);
        k_far_adjoint<<<grid, FE_TILE, 0, s>>>(dd.as<double>(), nd, (const cx<double> *)G, A.spts.as<double>(),
                                               A.snrm.as<double>(), A.sw.as<double>(), A.perm.as<int32_t>(), pb->n,
                                               pb->nu, pb->ibc ? 1 : 0, A.k_re, A.k_im, pb->cibc,
                                               (cx<double> *)xbar);
        FMB_LAUNCH_CHECK();
        FMB_CHECK_HIP(hipStreamSynchronize(s));
    });
}

int bem_field_fmm(fmb_problem_t pb, const void *x, int32_t nrhs, const double *points, int64_t nt, int32_t region,
                  int32_t order, void *E, void *stream) {
    return guarded([&] {
        FMB_REQUIRE(pb && x && points && E, "bad arguments");
        FMB_REQUIRE(nrhs >= 1 && nrhs <= pb->nrhs_max, "nrhs out of range");
        FMB_REQUIRE(nt >= 1, "no target points");
        FMB_REQUIRE(region == 0 || (region == 1 && !pb->ibc && pb->J == 1),
                    "region must be 0 (host) or 1 (interior of a one-scatterer dielectric problem)");
        FMB_REQUIRE(order >= 1 && order <= MAX_ORDER, "order must be in [1, 24]");
        for (int64_t i = 0; i < 3 * nt; ++i) FMB_REQUIRE(std::isfinite(points[i]), "non-finite target point");
        hipStream_t s = (hipStream_t)stream;
        const Plan &A = pb->p0->p;
        const Plan &K = region == 1 ? pb->p1->p : A;
        const int64_t n = pb->n, m = n + nt;
        std::vector<double> sp(3 * n), sn(3 * n), sw(n);
        std::vector<int32_t> perm(n);
        FMB_CHECK_HIP(hipMemcpyAsync(sp.data(), A.spts.p, sp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipMemcpyAsync(sn.data(), A.snrm.p, sn.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipMemcpyAsync(sw.data(), A.sw.p, sw.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipMemcpyAsync(perm.data(), A.perm.p, perm.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        FMB_CHECK_HIP(hipStreamSynchronize(s));
        // nodes in user order, then the targets (unit normal, unit weight, zero density)
        std::vector<double> up(3 * m), un(3 * m), uw(m);
        for (int64_t i = 0; i < n; ++i) {
            const int64_t u = perm[i];
            for (int q = 0; q < 3; ++q) {
                up[3 * u + q] = sp[3 * i + q];
                un[3 * u + q] = sn[3 * i + q];
            }
            uw[u] = sw[i];
        }
        for (int64_t t = 0; t < nt; ++t) {
            for (int q = 0; q < 3; ++q) up[3 * (n + t) + q] = points[3 * t + q];
            un[3 * (n + t)] = un[3 * (n + t) + 1] = 0.0;
            un[3 * (n + t) + 2] = 1.0;
            uw[n + t] = 1.0;
        }
        fmb_plan_opts o;
        fmb_plan_opts_default(&o);
        o.precision = FMB_FP64;
        o.nrhs_max = nrhs;
        o.corr_mode = FMB_CORR_NONE;
        fmb_plan_t fp = nullptr;
        int rc = fmm_plan(up.data(), un.data(), uw.data(), m, K.k_re, K.k_im, order, &o, stream, &fp);
        if (rc != FMB_OK) throw Status{rc, std::string("field plan over nodes and targets: ") + fmb_last_error()};
        std::unique_ptr<fmb_plan_s, int (*)(fmb_plan_t)> own(fp, fmm_plan_destroy);
        DevBuf da, db, dy;
        const size_t bytes = (size_t)nrhs * m * 3 * sizeof(cx<double>);
        da.alloc(bytes);
        db.alloc(bytes);
        dy.alloc(bytes);
        const cx<double> tc = cdiv(mk(1.0, 0.0) - pb->eps, pb->eps);
        k_field_dens<<<dim3((unsigned)((m + TPB - 1) / TPB), (unsigned)nrhs), TPB, 0, s>>>(
            A.snrm.as<double>(), A.perm.as<int32_t>(), (const cx<double> *)x, n, nt, pb->nu, region,
            pb->ibc ? 1 : 0, tc, pb->gamma, pb->cibc, da.as<cx<double>>(), db.as<cx<double>>());
        FMB_LAUNCH_CHECK();
        rc = fmm_matvec(fp, da.p, db.p, dy.p, nrhs, stream);
        if (rc != FMB_OK) throw Status{rc, std::string("field product: ") + fmb_last_error()};
        k_field_take<<<dim3((unsigned)((nt + TPB - 1) / TPB), (unsigned)nrhs), TPB, 0, s>>>(
            dy.as<cx<double>>(), n, nt, region == 0 ? -1.0 : 1.0, (cx<double> *)E);
        FMB_LAUNCH_CHECK();
        FMB_CHECK_HIP(hipStreamSynchronize(s));
    });
}

int bem_problem_use_graphs(fmb_problem_t pb, int32_t enable) {
    return guarded([&] {
        FMB_REQUIRE(pb != nullptr, "problem is NULL");
        pb->graphs = enable != 0;
    });
}

int bem_apply(fmb_problem_t pb, const void *x, void *r, int32_t nrhs, void *stream) {
    return guarded([&] {
        FMB_REQUIRE(pb && x && r && x != r, "bad arguments");
        FMB_REQUIRE(nrhs >= 1 && nrhs <= pb->nrhs_max, "nrhs out of range");
        bem_apply_t<double>(*pb, (const cx<double> *)x, (cx<double> *)r, nrhs, (hipStream_t)stream);
    });
}

int bem_apply32(fmb_problem_t pb, const void *x, void *r, int32_t nrhs, void *stream) {
    return guarded([&] {
        FMB_REQUIRE(pb && x && r && x != r, "bad arguments");
        FMB_REQUIRE(pb->p032 != nullptr, "bem_apply32 needs the FP32 plans");
        FMB_REQUIRE(nrhs >= 1 && nrhs <= pb->nrhs_max, "nrhs out of range");
        bem_apply_t<float>(*pb, (const cx<float> *)x, (cx<float> *)r, nrhs, (hipStream_t)stream);
    });
}

int bem_apply_adjoint(fmb_problem_t pb, const void *x, void *r, int32_t nrhs, void *stream) {
    return guarded([&] {
        FMB_REQUIRE(pb && x && r && x != r, "bad arguments");
        FMB_REQUIRE(nrhs >= 1 && nrhs <= pb->nrhs_max, "nrhs out of range");
        bem_apply_adjoint_t<double>(*pb, (const cx<double> *)x, (cx<double> *)r, nrhs, (hipStream_t)stream, nullptr);
    });
}

int bem_precond_apply(fmb_problem_t pb, const void *v, void *z, int32_t nrhs, void *stream) {
    return guarded([&] {
        FMB_REQUIRE(pb && v && z, "bad arguments");
        FMB_REQUIRE(nrhs >= 1 && nrhs <= pb->nrhs_max, "nrhs out of range");
        precond_t<double>(*pb, (const cx<double> *)v, (cx<double> *)z, nrhs, (hipStream_t)stream);
    });
}

int bem_rhs_planewave(fmb_problem_t pb, const double *dirs, const double *pols, void *rhs, int32_t nrhs,
                      void *stream) {
    return guarded([&] {
        FMB_REQUIRE(pb && dirs && pols && rhs, "bad arguments");
        FMB_REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        hipStream_t s = (hipStream_t)stream;
        DevBuf dd, dp;
        dd.alloc(nrhs * 3 * sizeof(double));
        dp.alloc(nrhs * 3 * sizeof(cx<double>));
        FMB_CHECK_HIP(hipMemcpyAsync(dd.p, dirs, nrhs * 3 * sizeof(double), hipMemcpyHostToDevice, s));
        FMB_CHECK_HIP(hipMemcpyAsync(dp.p, pols, nrhs * 3 * sizeof(cx<double>), hipMemcpyHostToDevice, s));
        const Plan &A = pb->p0->p;
        k_rhs_planewave<<<gridn(pb->n * nrhs), TPB, 0, s>>>(A.spts.as<double>(), A.iperm.as<int32_t>(), dd.as<double>(),
                                                            dp.as<cx<double>>(), pb->n, nrhs, pb->k0_re, pb->k0_im, pb->nu,
                                                            (cx<double> *)rhs);
        FMB_LAUNCH_CHECK();
        FMB_CHECK_HIP(hipStreamSynchronize(s));
    });
}

int gmres_solve(fmb_problem_t pb, const void *rhs, void *x, int32_t nrhs, const fmb_gmres_opts *o,
                fmb_gmres_info *info, void *stream) {
    bool converged = true;
    const int code = guarded([&] {
        const fmb_gmres_opts op = solve_opts(o);
        converged = solve_one(pb, rhs, x, nrhs, op, info, (hipStream_t)stream);
    });
    if (code != FMB_OK) return code;
    if (!converged) {
        set_error("fGMRES reached maxit before the tolerance");
        return FMB_ENOCONV;
    }
    return FMB_OK;
}

int gmres_solve_group(const fmb_problem_t *pbs, int32_t count, const void *const *rhs, void *const *x,
                      const int32_t *nrhs, const fmb_gmres_opts *o, fmb_gmres_info *info, void *stream) {
    std::vector<int> codes;
    std::vector<std::string> msgs;
    std::vector<char> conv;
    const int code = guarded([&] {
        FMB_REQUIRE(pbs && rhs && x && nrhs && count >= 1, "bad arguments");
        const fmb_gmres_opts op = solve_opts(o);
        for (int i = 0; i < count; ++i) {
            check_solve_args(pbs[i], rhs[i], x[i], nrhs[i], op);
            for (int q = 0; q < i; ++q) {
                FMB_REQUIRE(pbs[q] != pbs[i], "a problem appears twice in the group");
                const fmb_problem_s &A = *pbs[q], &B = *pbs[i];
                std::vector<const fmb_plan_s *> pa = {A.p0, A.p032}, pbv = {B.p0, B.p032};
                for (int j = 0; j < A.J; ++j) pa.insert(pa.end(), {A.pj[j], A.pj32[j]});
                for (int j = 0; j < B.J; ++j) pbv.insert(pbv.end(), {B.pj[j], B.pj32[j]});
                for (const fmb_plan_s *x1 : pa)
                    for (const fmb_plan_s *x2 : pbv)
                        FMB_REQUIRE(!x1 || x1 != x2, "two problems of the group share a plan");
            }
        }
        int dev = 0;
        FMB_CHECK_HIP(hipGetDevice(&dev));
        hipStream_t cs = (hipStream_t)stream;
        hipEvent_t start = nullptr;
        FMB_CHECK_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
        struct EvFree {
            hipEvent_t e;
            ~EvFree() { (void)hipEventDestroy(e); }
        } start_free{start};
        FMB_CHECK_HIP(hipEventRecord(start, cs));
        codes.assign(count, FMB_OK);
        msgs.assign(count, std::string());
        conv.assign(count, 1);
        // one host thread and one stream per problem: the problems' launches
        // overlap on the GPU while each solve keeps its own host decisions
        std::vector<std::thread> th;
        th.reserve(count);
        for (int i = 0; i < count; ++i) {
            th.emplace_back([&, i] {
                hipStream_t si = nullptr;
                codes[i] = guarded([&] {
                    FMB_CHECK_HIP(hipSetDevice(dev));
                    FMB_CHECK_HIP(hipStreamCreateWithFlags(&si, hipStreamNonBlocking));
                    FMB_CHECK_HIP(hipStreamWaitEvent(si, start, 0));
                    conv[i] = solve_one(pbs[i], rhs[i], x[i], nrhs[i], op, info ? info + i : nullptr, si) ? 1 : 0;
                    FMB_CHECK_HIP(hipStreamSynchronize(si));
                });
                if (codes[i] != FMB_OK) {
                    msgs[i] = fmb_last_error();
                    if (si) (void)hipStreamSynchronize(si);
                }
                if (si) (void)hipStreamDestroy(si);
            });
        }
        for (auto &t : th) t.join();
        for (int i = 0; i < count; ++i)
            if (codes[i] != FMB_OK)
                throw Status{codes[i], "problem " + std::to_string(i) + " of the group: " + msgs[i]};
    });
    if (code != FMB_OK) return code;
    for (int i = 0; i < count; ++i)
        if (!conv[i]) {
            set_error("fGMRES reached maxit before the tolerance (problem " + std::to_string(i) + " of the group)");
            return FMB_ENOCONV;
        }
    return FMB_OK;
}

int bem_problem_destroy(fmb_problem_t pb) {
    return guarded([&] { delete pb; });
}

}  // extern "C"
