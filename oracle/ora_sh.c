/*
 * Real spherical harmonics from their definition. TEST INFRASTRUCTURE ONLY.
 *
 * The paper gives each Gaussian a "color c" (Sec. 3); view-dependent colour is
 * read here as real spherical harmonics of degree <= 3 evaluated on the unit
 * direction from the camera centre to the Gaussian mean, plus 0.5, clamped at 0.
 *
 * Definition used (orthonormal real SH with the Condon-Shortley phase, index
 * k = l^2 + l + m, m = -l..l):
 *   Y_l^0  = K_l^0 P_l^0(z)
 *   Y_l^m  = sqrt(2) K_l^m cos(m phi) P_l^m(z)        (m > 0)
 *   Y_l^-m = sqrt(2) K_l^m sin(m phi) P_l^m(z)        (m > 0)
 *   K_l^m  = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)
 *   P_l^m(z) = (-1)^m (1-z^2)^(m/2) d^m/dz^m P_l(z),  P_l the Legendre polynomial.
 * On the unit sphere sin^m(theta) cos(m phi) = Re((x+iy)^m) and
 * sin^m(theta) sin(m phi) = Im((x+iy)^m), so each Y is a polynomial in (x,y,z);
 * its gradient with respect to (x,y,z) is returned as well.
 */
#include <math.h>
#include <string.h>

#include "ora.h"

#define ORA_SH_MAXL 8

int ora_sh_count(int degree) { return (degree + 1) * (degree + 1); }

/* coefficients (ascending powers) of the Legendre polynomials P_0..P_L (Bonnet recurrence) */
static void legendre_coeffs(int L, double c[ORA_SH_MAXL + 1][ORA_SH_MAXL + 1])
{
    memset(c, 0, sizeof(double) * (ORA_SH_MAXL + 1) * (ORA_SH_MAXL + 1));
    c[0][0] = 1.0;
    if (L >= 1) c[1][1] = 1.0;
    for (int n = 1; n < L; ++n) {
        /* (n+1) P_{n+1} = (2n+1) z P_n - n P_{n-1} */
        for (int k = 0; k <= n + 1; ++k) {
            double v = 0.0;
            if (k >= 1) v += (2.0 * n + 1.0) * c[n][k - 1];
            v -= n * c[n - 1][k];
            c[n + 1][k] = v / (n + 1.0);
        }
    }
}

/* value of the m-th derivative of the polynomial with coefficients p (degree <= L) at z */
static double poly_deriv(const double* p, int L, int m, double z)
{
    double s = 0.0;
    for (int k = L; k >= m; --k) {
        double f = 1.0;
        for (int j = 0; j < m; ++j) f *= (double)(k - j);
        s = s * z + f * p[k];
    }
    /* Horner above accumulates powers z^(k-m) for k from L down to m */
    return s;
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

void ora_sh_basis(int degree, const double d[3], double* Y, double* dY)
{
    double leg[ORA_SH_MAXL + 1][ORA_SH_MAXL + 1];
    int L = degree;
    legendre_coeffs(L, leg);
    const double x = d[0], y = d[1], z = d[2];
    /* A_m = Re((x+iy)^m), B_m = Im((x+iy)^m) */
    double A[ORA_SH_MAXL + 2], B[ORA_SH_MAXL + 2];
    A[0] = 1.0;
    B[0] = 0.0;
    for (int m = 1; m <= L; ++m) {
        A[m] = x * A[m - 1] - y * B[m - 1];
        B[m] = x * B[m - 1] + y * A[m - 1];
    }
    for (int l = 0; l <= L; ++l) {
        for (int m = 0; m <= l; ++m) {
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - m) / factorial(l + m));
            double sgn = (m % 2) ? -1.0 : 1.0; /* Condon-Shortley phase */
            double Pm = poly_deriv(leg[l], l, m, z);       /* d^m P_l / dz^m */
            double Pm1 = (m + 1 <= l) ? poly_deriv(leg[l], l, m + 1, z) : 0.0;
            if (m == 0) {
                int k = l * l + l;
                Y[k] = K * Pm;
                if (dY) {
                    dY[3 * k + 0] = 0.0;
                    dY[3 * k + 1] = 0.0;
                    dY[3 * k + 2] = K * Pm1;
                }
            } else {
                double f = sqrt(2.0) * K * sgn;
                int kp = l * l + l + m, kn = l * l + l - m;
                Y[kp] = f * A[m] * Pm;
                Y[kn] = f * B[m] * Pm;
                if (dY) {
                    /* dA_m/dx = m A_{m-1}, dA_m/dy = -m B_{m-1}; dB_m/dx = m B_{m-1}, dB_m/dy = m A_{m-1} */
                    dY[3 * kp + 0] = f * m * A[m - 1] * Pm;
                    dY[3 * kp + 1] = f * (-m) * B[m - 1] * Pm;
                    dY[3 * kp + 2] = f * A[m] * Pm1;
                    dY[3 * kn + 0] = f * m * B[m - 1] * Pm;
                    dY[3 * kn + 1] = f * m * A[m - 1] * Pm;
                    dY[3 * kn + 2] = f * B[m] * Pm1;
                }
            }
        }
    }
}
