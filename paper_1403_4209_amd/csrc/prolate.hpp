// The prolate spheroidal taper psi_0(c, x), c = 3*pi (the gridding function's image-plane
// form): expansion in normalised Legendre polynomials whose coefficients are the eigenvector
// of the (even-index) tridiagonal matrix of the spheroidal differential operator for its
// smallest eigenvalue (Bouwkamp's method; Xiao, Rokhlin & Yarvin 2001). Used by the kernel
// table build and by the image finaliser's taper correction.
#pragma once

#include <math.h>

#include <hip/hip_runtime.h>

namespace wg {

constexpr int kTaperTerms = 40;
constexpr double kTaperC = 3.0 * M_PI;

struct TaperCoef {
    int n;
    double c[kTaperTerms];  // psi_0(x) = sum_i c[i] * P_{2i}(x)
};

// Coefficients of psi_0(c, .), normalised to unit L2 norm on [-1, 1] and psi_0(c, 0) > 0 (host).
void prolate_coefficients(double c, TaperCoef *tc);

// psi_0(c, x) for |x| < 1 and 0 outside the open field of view.
__device__ inline double taper(double x, const TaperCoef &tc) {
#pragma clang fp contract(off)
    if (!(fabs(x) < 1.0)) return 0.0;
    double pm = 1.0, pc = x, s = tc.c[0];
    for (int m = 1; m < 2 * tc.n - 1; ++m) {
        double pn = ((2.0 * m + 1.0) * x * pc - (double)m * pm) / (double)(m + 1);
        pm = pc;
        pc = pn;
        if (((m + 1) & 1) == 0) s += tc.c[(m + 1) >> 1] * pc;
    }
    return s;
}

}  // namespace wg
