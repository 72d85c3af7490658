// Basis evaluation shared by the forward and adjoint expansion kernels:
// normalised associated Legendre recurrences and the regular solid harmonics
// R_n^m(d) = j_n(k|d|) Y_n^m(d/|d|) (eqs. 2.14-2.15), with constants tabulated
// on the host at plan time.
#pragma once
#include "common.h"

namespace fmb {

// ---------------------------------------------------------------- basis
// Recurrence constants of the normalised associated Legendre functions and of
// the gradient of R_n^m, tabulated on the host at plan time (BasisTab layout
// below) so that the per-node loops carry no square roots or divisions.
//   Q_m^m = qmm[m],  Q_{m+1}^m = q1[m] x Q_m^m,
//   Q_n^m = la[n][m] (x Q_{n-1}^m - lb[n][m] Q_{n-2}^m)            (n >= m + 2)
template <typename T>
struct BasisTab {
    const T *la, *lb, *qmm, *q1;     // [(N+1)^2] (row n, column m), [(N+1)^2], [N+1], [N+1]
    const T *gco;                    // [P2][6] gradient coefficients of coefficient idx (mu = -m)
    const int32_t *gix;              // [P2][7] R-table indices of the six gradient terms and of R_n^{-m}
    int N;
};

template <typename T>
__device__ inline BasisTab<T> basis_tab(const T *tab, const int32_t *gix, int N, int P2) {
    BasisTab<T> b;
    const int NN = (N + 1) * (N + 1);
    b.la = tab;
    b.lb = tab + NN;
    b.qmm = tab + 2 * NN;
    b.q1 = tab + 2 * NN + (N + 1);
    b.gco = tab + 2 * NN + 2 * (N + 1);
    b.gix = gix;
    b.N = N;
    (void)P2;
    return b;
}

// R_n^m(d) for n <= N, one order m, of one point into out[(N+1)^2]; jb holds
// j_0..j_N at k|d|.
// x = cos th, w = sin th e^{i ph} of the point's direction from the centre.
template <typename T>
__device__ inline void regular_column(T x, cx<T> w, const cx<T> *jb, const BasisTab<T> &bt, int m, cx<T> *out) {
    const int N = bt.N;
    const T qmm = bt.qmm[m];
    cx<T> wm = mk(T(1), T(0));
    for (int i = 1; i <= m; ++i) wm = wm * w;
    const T sgn = (m & 1) ? T(-1) : T(1);
    T q2 = 0, q1 = qmm;
    for (int n = m; n <= N; ++n) {
        T q;
        if (n == m) q = qmm;
        else if (n == m + 1) q = bt.q1[m] * x * qmm;
        else q = bt.la[n * (N + 1) + m] * (x * q1 - bt.lb[n * (N + 1) + m] * q2);
        if (n > m) {
            q2 = q1;
            q1 = q;
        }
        cx<T> Y = (sgn * q) * wm;
        out[n * n + n + m] = jb[n] * Y;
        if (m > 0) out[n * n + n - m] = jb[n] * conj(Y);
    }
}

}  // namespace fmb
