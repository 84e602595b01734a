// Host construction of the sigma-point rules (Section 4.3): the 1-D
// Gauss-Hermite rule for N(0, 1) by the Golub-Welsch method (the nodes are
// the eigenvalues of the symmetric tridiagonal Jacobi matrix of the
// probabilists' Hermite recurrence He_{k+1} = x He_k - k He_{k-1}, found here
// with cyclic Jacobi rotations), polished by Newton steps on He_p, with the
// weights (p-1)! / (p He_{p-1}(x)^2) of the Gaussian probability measure.
#pragma once

#include <math.h>

namespace pss {

// He_{p-1}(x) and He_p(x)
inline void hermite_pair(int p, double x, double &hm1, double &hp)
{
    double a = 1.0, b = x; // He_0, He_1
    for (int k = 1; k < p; ++k) {
        const double c = x * b - k * a;
        a = b;
        b = c;
    }
    hm1 = a;
    hp = b;
}

// nodes x[0..p-1] (ascending) and weights w (summing to one); p in 2..20
inline void gauss_hermite_1d(int p, double *x, double *w)
{
    double A[20][20] = {};
    for (int k = 1; k < p; ++k)
        A[k - 1][k] = A[k][k - 1] = sqrt((double)k);
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < p; ++i)
            for (int j = i + 1; j < p; ++j)
                off += A[i][j] * A[i][j];
        if (off < 1e-30)
            break;
        for (int i = 0; i < p; ++i)
            for (int j = i + 1; j < p; ++j) {
                if (fabs(A[i][j]) < 1e-300)
                    continue;
                // rotation in the (i, j) plane that zeroes A[i][j]
                const double th = (A[j][j] - A[i][i]) / (2.0 * A[i][j]);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < p; ++k) {
                    const double aki = A[k][i], akj = A[k][j];
                    A[k][i] = c * aki - s * akj;
                    A[k][j] = s * aki + c * akj;
                }
                for (int k = 0; k < p; ++k) {
                    const double aik = A[i][k], ajk = A[j][k];
                    A[i][k] = c * aik - s * ajk;
                    A[j][k] = s * aik + c * ajk;
                }
            }
    }
    for (int i = 0; i < p; ++i)
        x[i] = A[i][i];
    for (int i = 1; i < p; ++i) // insertion sort
        for (int j = i; j > 0 && x[j - 1] > x[j]; --j) {
            const double t = x[j];
            x[j] = x[j - 1];
            x[j - 1] = t;
        }
    double fact = 1.0; // (p-1)!
    for (int k = 2; k < p; ++k)
        fact *= k;
    double sum = 0.0;
    for (int i = 0; i < p; ++i) {
        double hm1, hp;
        for (int it = 0; it < 3; ++it) { // He_p' = p He_{p-1}
            hermite_pair(p, x[i], hm1, hp);
            x[i] -= hp / (p * hm1);
        }
        hermite_pair(p, x[i], hm1, hp);
        w[i] = fact / (p * hm1 * hm1);
        sum += w[i];
    }
    // exact symmetry of the rule, weights normalised to sum one
    for (int i = 0; i < p / 2; ++i) {
        const double xs = 0.5 * (x[p - 1 - i] - x[i]), ws = 0.5 * (w[i] + w[p - 1 - i]);
        x[i] = -xs;
        x[p - 1 - i] = xs;
        w[i] = w[p - 1 - i] = ws;
    }
    if (p % 2)
        x[p / 2] = 0.0;
    for (int i = 0; i < p; ++i)
        w[i] /= sum;
}

} // namespace pss
