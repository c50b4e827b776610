// Eigenvalues of a small real upper Hessenberg matrix (the Ritz values that set the Newton
// basis shifts) and their Leja ordering.  Written for one thread of a workgroup; also
// callable from host code.
//
// The eigenvalues come from the implicitly shifted double-shift QR iteration of Francis
// (Golub and Van Loan, Matrix Computations, Section 7.5): on the active unreduced block
// [lo, hi], the two shifts are the eigenvalues of its trailing 2 x 2 block (a real
// polynomial s = trace, t = determinant), the first column of (H - s1)(H - s2) is reduced by
// a 3 x 3 Householder reflector, and the resulting bulge is chased down the subdiagonal.  A
// subdiagonal entry below eps times its neighbouring diagonal entries is set to zero, which
// splits the problem; 1 x 1 and 2 x 2 blocks give the eigenvalues directly.  After every ten
// iterations without a split an exceptional shift pair is used.  Only the active block is
// updated (no Schur vectors are needed).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace sko {

struct Eig2 {
    double re0, im0, re1, im1;
};

// Eigenvalues of [[a, b], [c, d]].
__host__ __device__ inline Eig2 eig2x2(double a, double b, double c, double d) {
    const double m = 0.5 * (a + d), p = 0.5 * (a - d);
    const double disc = p * p + b * c;
    Eig2 e{};
    if (disc >= 0.0) {
        const double r = sqrt(disc);
        // larger-magnitude root first, the other from the determinant (no cancellation)
        const double l0 = m + (m >= 0.0 ? r : -r);
        const double det = a * d - b * c;
        e.re0 = l0;
        e.re1 = l0 != 0.0 ? det / l0 : m - (m >= 0.0 ? r : -r);
        e.im0 = e.im1 = 0.0;
    } else {
        const double r = sqrt(-disc);
        e.re0 = e.re1 = m;
        e.im0 = r;
        e.im1 = -r;
    }
    return e;
}

// H: n x n upper Hessenberg, column-major with leading dimension ld, overwritten.  wr, wi:
// real and imaginary parts (complex pairs adjacent, positive imaginary part first).
// Returns false when an eigenvalue took more than 60 iterations.
__host__ __device__ inline bool hessenberg_eigenvalues(double* H, int n, int ld, double* wr, double* wi) {
    auto at = [&](int i, int j) -> double& { return H[i + (long)j * ld]; };
    const double eps = 2.220446049250313e-16;
    double fro = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= (j + 1 < n ? j + 1 : n - 1); ++i) fro += at(i, j) * at(i, j);
    fro = sqrt(fro);
    int hi = n - 1, iter = 0;
    while (hi >= 0) {
        int lo = hi;
        while (lo > 0) {
            double scale = fabs(at(lo - 1, lo - 1)) + fabs(at(lo, lo));
            if (scale == 0.0) scale = fro;
            if (fabs(at(lo, lo - 1)) <= eps * scale) {
                at(lo, lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            wr[hi] = at(hi, hi);
            wi[hi] = 0.0;
            --hi;
            iter = 0;
            continue;
        }
        if (lo == hi - 1) {
            const Eig2 e = eig2x2(at(hi - 1, hi - 1), at(hi - 1, hi), at(hi, hi - 1), at(hi, hi));
            wr[hi - 1] = e.re0;
            wi[hi - 1] = e.im0;
            wr[hi] = e.re1;
            wi[hi] = e.im1;
            hi -= 2;
            iter = 0;
            continue;
        }
        if (++iter > 60) return false;
        double s, t;
        if (iter % 10 == 0) {
            // exceptional pair x +- i e from the size of the last two subdiagonal entries
            const double e = fabs(at(hi, hi - 1)) + fabs(at(hi - 1, hi - 2));
            const double x = at(hi, hi) + 0.5 * e;
            s = 2.0 * x;
            t = x * x + e * e;
        } else {
            const double a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
            s = a + d;
            t = a * d - b * c;
        }
        // first column of H^2 - s H + t I on the active block
        double x = at(lo, lo) * at(lo, lo) + at(lo, lo + 1) * at(lo + 1, lo) - s * at(lo, lo) + t;
        double y = at(lo + 1, lo) * (at(lo, lo) + at(lo + 1, lo + 1) - s);
        double z = at(lo + 1, lo) * at(lo + 2, lo + 1);
        for (int k = lo; k <= hi - 1; ++k) {
            const int len = (k <= hi - 2) ? 3 : 2;
            double u0 = x, u1 = y, u2 = len == 3 ? z : 0.0;
            const double nrm = sqrt(u0 * u0 + u1 * u1 + u2 * u2);
            if (nrm != 0.0) {
                const double alpha = u0 >= 0.0 ? -nrm : nrm;
                const double v0 = u0 - alpha, v1 = u1, v2 = u2;
                const double beta = 2.0 / (v0 * v0 + v1 * v1 + v2 * v2);
                // from the left: rows k..k+len-1, columns max(lo, k-1)..hi
                for (int j = (k > lo ? k - 1 : lo); j <= hi; ++j) {
                    double d = v0 * at(k, j) + v1 * at(k + 1, j);
                    if (len == 3) d += v2 * at(k + 2, j);
                    d *= beta;
                    at(k, j) -= d * v0;
                    at(k + 1, j) -= d * v1;
                    if (len == 3) at(k + 2, j) -= d * v2;
                }
                if (k > lo) {  // the bulge column is now reduced
                    at(k + 1, k - 1) = 0.0;
                    if (len == 3) at(k + 2, k - 1) = 0.0;
                }
                // from the right: columns k..k+len-1, rows lo..min(k+3, hi)
                const int rmax = (k + 3 < hi) ? k + 3 : hi;
                for (int i = lo; i <= rmax; ++i) {
                    double d = at(i, k) * v0 + at(i, k + 1) * v1;
                    if (len == 3) d += at(i, k + 2) * v2;
                    d *= beta;
                    at(i, k) -= d * v0;
                    at(i, k + 1) -= d * v1;
                    if (len == 3) at(i, k + 2) -= d * v2;
                }
            }
            if (k <= hi - 2) {
                x = at(k + 1, k);
                y = at(k + 2, k);
                if (k <= hi - 3) z = at(k + 3, k);
            }
        }
    }
    return true;
}

// Leja ordering of the eigenvalues (wr, wi) and the Newton recurrence coefficients of s
// steps: v_{j+1} = (A - a_j) v_j + b_j v_{j-1}.  Candidates are the eigenvalues with wi >= 0
// sorted by (real, imaginary part); the first is the one of largest modulus, each next one
// maximises the sum of log distances to the points chosen so far (conjugates included),
// the first maximum in the sorted order winning; a complex point brings its conjugate.  A
// real shift theta gives (a, b) = (theta, 0); a complex pair alpha +- i beta two steps
// (alpha, 0), (alpha, beta^2), or, in the last step, (alpha, 0) alone.  cre/cim: n scratch
// entries each; a, b: s entries each (zero where the points run out).
__host__ __device__ inline void leja_newton_coefficients(const double* wr, const double* wi, int n, int s,
                                                         double* cre, double* cim, double* ore, double* oim,
                                                         double* a, double* b) {
    int nc = 0;
    for (int i = 0; i < n; ++i)
        if (wi[i] >= 0.0) {
            // insertion by (real, imaginary)
            int p = nc++;
            while (p > 0 && (cre[p - 1] > wr[i] || (cre[p - 1] == wr[i] && cim[p - 1] > wi[i]))) {
                cre[p] = cre[p - 1];
                cim[p] = cim[p - 1];
                --p;
            }
            cre[p] = wr[i];
            cim[p] = wi[i];
        }
    int no = 0;  // chosen points (with conjugates) in ore/oim
    for (int j = 0; j < s; ++j) a[j] = b[j] = 0.0;
    int j = 0;
    while (nc > 0 && j < s) {
        int best = 0;
        if (no == 0) {
            double bm = -1.0;
            for (int i = 0; i < nc; ++i) {
                const double m = hypot(cre[i], cim[i]);
                if (m > bm) {
                    bm = m;
                    best = i;
                }
            }
        } else {
            double bs = -INFINITY;
            bool first = true;
            for (int i = 0; i < nc; ++i) {
                double sc = 0.0;
                for (int q = 0; q < no; ++q) {
                    const double d = hypot(cre[i] - ore[q], cim[i] - oim[q]);
                    if (d == 0.0) {
                        sc = -INFINITY;
                        break;
                    }
                    sc += log(d);
                }
                if (first || sc > bs) {
                    bs = sc;
                    best = i;
                    first = false;
                }
            }
        }
        const double zr = cre[best], zi = cim[best];
        for (int i = best; i + 1 < nc; ++i) {
            cre[i] = cre[i + 1];
            cim[i] = cim[i + 1];
        }
        --nc;
        ore[no] = zr;
        oim[no] = zi;
        ++no;
        if (zi > 0.0) {
            ore[no] = zr;
            oim[no] = -zi;
            ++no;
            a[j] = zr;
            if (j + 1 < s) {
                a[j + 1] = zr;
                b[j + 1] = zi * zi;
                j += 2;
            } else {
                j += 1;
            }
        } else {
            a[j] = zr;
            j += 1;
        }
    }
}

}  // namespace sko
