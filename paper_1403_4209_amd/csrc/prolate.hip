// Host computation of the prolate spheroidal expansion coefficients (see prolate.hpp).
#include <math.h>

#include "prolate.hpp"

#pragma clang fp contract(off)

namespace wg {


// Smallest-eigenvalue eigenvector of the symmetric tridiagonal matrix of the operator
// -((1-x^2)psi')' + c^2 x^2 psi in the basis sqrt(k+1/2) P_k, k even: the eigenvalue by
// bisection on the Sturm count, the eigenvector by inverse iteration (banded Gaussian
// elimination with partial pivoting).
void prolate_coefficients(double c, TaperCoef *tc) {
    const int K = kTaperTerms;
    double d[kTaperTerms], e[kTaperTerms];
    auto a = [](double k) { return (k + 1.0) / sqrt((2.0 * k + 1.0) * (2.0 * k + 3.0)); };
    for (int i = 0; i < K; ++i) {
        const double k = 2.0 * i;
        d[i] = k * (k + 1.0) + c * c * (a(k) * a(k) + (i > 0 ? a(k - 1.0) * a(k - 1.0) : 0.0));
        e[i] = (i + 1 < K) ? c * c * a(k) * a(k + 1.0) : 0.0;
    }
    double lo = d[0], hi = d[0];
    for (int i = 0; i < K; ++i) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < K ? fabs(e[i]) : 0.0);
        lo = fmin(lo, d[i] - r);
        hi = fmax(hi, d[i] + r);
    }
    auto count_below = [&](double x) {
        int cnt = 0;
        double q = 1.0;
        for (int i = 0; i < K; ++i) {
            q = d[i] - x - (i > 0 ? e[i - 1] * e[i - 1] / q : 0.0);
            if (q == 0.0) q = -1e-300;
            if (q < 0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * fmax(1.0, fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count_below(mid) >= 1)
            hi = mid;
        else
            lo = mid;
    }
    const double lam = 0.5 * (lo + hi);
    double v[kTaperTerms];
    for (int i = 0; i < K; ++i) v[i] = 1.0;
    for (int iter = 0; iter < 4; ++iter) {
        double A[kTaperTerms][3], b[kTaperTerms], sub[kTaperTerms], x[kTaperTerms];
        for (int i = 0; i < K; ++i) {
            A[i][0] = d[i] - lam;
            A[i][1] = (i + 1 < K) ? e[i] : 0.0;
            A[i][2] = 0.0;
            sub[i] = (i > 0) ? e[i - 1] : 0.0;
            b[i] = v[i];
        }
        for (int i = 0; i < K - 1; ++i) {
            if (fabs(sub[i + 1]) > fabs(A[i][0])) {  // swap rows i and i+1, then eliminate
                const double r0 = sub[i + 1], r1 = A[i + 1][0], r2 = A[i + 1][1], rb = b[i + 1];
                const double s0 = A[i][0], s1 = A[i][1], s2 = A[i][2], sb = b[i];
                A[i][0] = r0;
                A[i][1] = r1;
                A[i][2] = r2;
                b[i] = rb;
                const double f = s0 / r0;
                A[i + 1][0] = s1 - f * r1;
                A[i + 1][1] = s2 - f * r2;
                b[i + 1] = sb - f * rb;
            } else {
                const double f = sub[i + 1] / A[i][0];
                A[i + 1][0] -= f * A[i][1];
                A[i + 1][1] -= f * A[i][2];
                b[i + 1] -= f * b[i];
            }
        }
        for (int i = K - 1; i >= 0; --i) {
            double sacc = b[i];
            if (i + 1 < K) sacc -= A[i][1] * x[i + 1];
            if (i + 2 < K) sacc -= A[i][2] * x[i + 2];
            const double piv = A[i][0] == 0.0 ? 1e-300 : A[i][0];
            x[i] = sacc / piv;
        }
        double nrm = 0.0;
        for (int i = 0; i < K; ++i) nrm += x[i] * x[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < K; ++i) v[i] = x[i] / nrm;
    }
    // psi(0) = sum c_i P_{2i}(0), P_{2i}(0) = (-1)^i (2i-1)!!/(2i)!!
    double p0 = 1.0, psi0 = 0.0;
    for (int i = 0; i < K; ++i) {
        tc->c[i] = v[i] * sqrt(2.0 * i + 0.5);
        psi0 += tc->c[i] * p0;
        p0 *= -(2.0 * i + 1.0) / (2.0 * i + 2.0);
    }
    if (psi0 < 0)
        for (int i = 0; i < K; ++i) tc->c[i] = -tc->c[i];
    tc->n = K;
}

}  // namespace wg
