// smoothing.cpp -- coefficients of the smoothing polynomial p_r of Eq. (35).
//
// p_r has degree <= r + 1, p_r(-1) = 1, p_r(1) = 0 and its first r moments on [-1, 1]
// equal those of the step theta (Sec. 5.1). Writing p_r(s) = int_s^1 K(t) dt, these
// conditions say K has degree <= r, int K = 1 and int t^i K = 0 for i = 1..r: K is the
// reproducing kernel at 0 of the polynomials of degree <= r in L2(-1, 1),
//     K(t) = sum_{n=0}^{r} (2n + 1)/2 P_n(0) P_n(t)   (Legendre polynomials P_n).
// Everything is computed in exact rational arithmetic and rounded once to double.
#include <cstdint>
#include <cstdlib>

#include "host_common.hpp"

namespace ldm {

namespace {

using i128 = __int128;

i128 gcd128(i128 a, i128 b) {
    if (a < 0) a = -a;
    if (b < 0) b = -b;
    while (b != 0) {
        i128 t = a % b;
        a = b;
        b = t;
    }
    return a;
}

struct Q {
    i128 n = 0, d = 1;
};

Q norm(Q q) {
    if (q.d < 0) {
        q.n = -q.n;
        q.d = -q.d;
    }
    i128 g = gcd128(q.n, q.d);
    if (g > 1) {
        q.n /= g;
        q.d /= g;
    }
    return q;
}

Q add(Q a, Q b) { return norm(Q{a.n * b.d + b.n * a.d, a.d * b.d}); }
Q mul(Q a, Q b) { return norm(Q{a.n * b.n, a.d * b.d}); }
Q qi(long long n, long long d = 1) { return norm(Q{(i128)n, (i128)d}); }

}  // namespace

int smoothing_coefficients(int r, double* coef) {
    if (r < 1 || r > 8) return -1;
    // Legendre coefficients, (n + 1) P_{n+1} = (2n + 1) t P_n - n P_{n-1}
    Q P[10][10];
    P[0][0] = qi(1);
    P[1][1] = qi(1);
    for (int n = 1; n < r; ++n) {
        for (int k = 0; k <= n + 1; ++k) {
            Q v = qi(0);
            if (k >= 1) v = add(v, mul(qi(2 * n + 1, n + 1), P[n][k - 1]));
            v = add(v, mul(qi(-n, n + 1), P[n - 1][k]));
            P[n + 1][k] = v;
        }
    }
    Q K[10];
    for (int k = 0; k <= r; ++k) K[k] = qi(0);
    for (int n = 0; n <= r; ++n) {
        const Q w = mul(qi(2 * n + 1, 2), P[n][0]);   // (2n + 1)/2 P_n(0)
        for (int k = 0; k <= n; ++k) K[k] = add(K[k], mul(w, P[n][k]));
    }
    // p(s) = int_s^1 K = sum_k K_k (1 - s^{k+1}) / (k + 1)
    Q c[10];
    for (int k = 0; k <= r + 1; ++k) c[k] = qi(0);
    for (int k = 0; k <= r; ++k) {
        const Q t = mul(K[k], qi(1, k + 1));
        c[0] = add(c[0], t);
        c[k + 1] = add(c[k + 1], mul(t, qi(-1)));
    }
    for (int k = 0; k <= r + 1; ++k) coef[k] = (double)(long long)c[k].n / (double)(long long)c[k].d;
    return 0;
}

}  // namespace ldm
