/* Oracle helper: successive over-relaxation (Gauss-Seidel for omega = 1) on a CSR matrix.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle, never linked by the product library.
 *
 * Plain lexicographic sweeps x_i <- (1-w) x_i + w (b_i - sum_{j != i} a_ij x_j) / a_ii, used
 * as an iteration independent of the direct band elimination.  The residual
 * ||b - A x||_2 / ||b||_2 is evaluated every `check_every` sweeps; the loop stops when it
 * is <= tol, when it stops decreasing over 20 checks (stagnation at round-off), or after
 * max_sweeps.  Returns the number of sweeps done; *rel_res receives the last residual.
 */
#include <math.h>
#include <stdint.h>

static double residual(int64_t n, const int64_t *ip, const int64_t *ix, const double *a,
                       const double *b, const double *x, double bnorm)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = b[i];
        for (int64_t k = ip[i]; k < ip[i + 1]; ++k) r -= a[k] * x[ix[k]];
        s += r * r;
    }
    return sqrt(s) / bnorm;
}

int64_t sor_csr(int64_t n, const int64_t *ip, const int64_t *ix, const double *a,
                const double *b, double *x, double omega, int64_t max_sweeps, double tol,
                int64_t check_every, double *rel_res)
{
    double bnorm = 0.0;
    for (int64_t i = 0; i < n; ++i) bnorm += b[i] * b[i];
    bnorm = sqrt(bnorm);
    if (bnorm == 0.0) bnorm = 1.0;
    double best = residual(n, ip, ix, a, b, x, bnorm);
    int64_t since_best = 0;
    int64_t sweep = 0;
    *rel_res = best;
    while (sweep < max_sweeps && *rel_res > tol) {
        for (int64_t i = 0; i < n; ++i) {
            double diag = 0.0, s = b[i];
            for (int64_t k = ip[i]; k < ip[i + 1]; ++k) {
                if (ix[k] == i) diag += a[k];
                else s -= a[k] * x[ix[k]];
            }
            x[i] = (1.0 - omega) * x[i] + omega * s / diag;
        }
        ++sweep;
        if (sweep % check_every == 0) {
            *rel_res = residual(n, ip, ix, a, b, x, bnorm);
            if (*rel_res < 0.999 * best) { best = *rel_res; since_best = 0; }
            else if (++since_best >= 20) break;
        }
    }
    *rel_res = residual(n, ip, ix, a, b, x, bnorm);
    return sweep;
}
