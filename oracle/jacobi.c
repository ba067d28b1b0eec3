/*
 * Cyclic Jacobi diagonalisation of a complex Hermitian matrix, FP64.
 *
 * TEST INFRASTRUCTURE ONLY: part of the CPU oracle.  Plain C, single-threaded,
 * no BLAS/LAPACK.  It diagonalises the dense plane-wave Hamiltonian of
 * sec. 2.1 (the projected eigenproblem with identity overlap) so that the
 * lowest eigenvalues can be compared with the block LOBPCG of sec. 3.2.
 *
 * Each 2x2 pivot [[a, b], [conj(b), d]] with b = |b| e^{i phi} is written as
 * D M D^H with D = diag(1, e^{-i phi}) and M = [[a, |b|], [|b|, d]] real; the
 * classical Jacobi rotation G = [[c, s], [-s, c]] diagonalises M, so
 * J = D G = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] diagonalises the pivot.
 * A <- J^H A J touches rows and columns p, q only; V <- V J accumulates the
 * eigenvectors.  Sweeps run over all p < q in row order until the
 * off-diagonal Frobenius norm falls below tol * ||A||_F.
 *
 * Storage: row-major, interleaved complex (re, im), n x n.
 */
#include <math.h>
#include <stddef.h>

#define RE(m, i, j) (m)[2 * ((size_t)(i) * n + (j))]
#define IM(m, i, j) (m)[2 * ((size_t)(i) * n + (j)) + 1]

static double offdiag2(int n, const double *a)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j) s += RE(a, i, j) * RE(a, i, j) + IM(a, i, j) * IM(a, i, j);
    return s;
}

/* Returns the number of sweeps used, or -1 if max_sweeps was reached. */
int jacobi_herm(int n, double *a, double *w, double *v, int max_sweeps, double tol)
{
    double fro2 = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            fro2 += RE(a, i, j) * RE(a, i, j) + IM(a, i, j) * IM(a, i, j);
    for (int i = 0; i < n; ++i) {
        IM(a, i, i) = 0.0;
        for (int j = 0; j < n; ++j) { RE(v, i, j) = (i == j); IM(v, i, j) = 0.0; }
    }
    int sweep = 0, done = 0;
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        if (offdiag2(n, a) <= tol * tol * fro2) { done = 1; break; }
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double br = RE(a, p, q), bi = IM(a, p, q);
                double babs = hypot(br, bi);
                double ap = RE(a, p, p), dq = RE(a, q, q);
                if (babs == 0.0) continue;
                if (babs < 1e-300 || babs <= 1e-18 * (fabs(ap) + fabs(dq))) {
                    RE(a, p, q) = IM(a, p, q) = RE(a, q, p) = IM(a, q, p) = 0.0;
                    continue;
                }
                double ph_r = br / babs, ph_i = bi / babs;     /* e^{i phi} */
                double tau = (dq - ap) / (2.0 * babs);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* e^{-i phi} = (ph_r, -ph_i) */
                /* columns: new_p = c A_p - s e^{-i phi} A_q ; new_q = s A_p + c e^{-i phi} A_q */
                for (int k = 0; k < n; ++k) {
                    double xr = RE(a, k, p), xi = IM(a, k, p);
                    double yr = RE(a, k, q), yi = IM(a, k, q);
                    double er = ph_r * yr + ph_i * yi;          /* e^{-i phi} * y */
                    double ei = ph_r * yi - ph_i * yr;
                    RE(a, k, p) = c * xr - s * er; IM(a, k, p) = c * xi - s * ei;
                    RE(a, k, q) = s * xr + c * er; IM(a, k, q) = s * xi + c * ei;
                    xr = RE(v, k, p); xi = IM(v, k, p);
                    yr = RE(v, k, q); yi = IM(v, k, q);
                    er = ph_r * yr + ph_i * yi;
                    ei = ph_r * yi - ph_i * yr;
                    RE(v, k, p) = c * xr - s * er; IM(v, k, p) = c * xi - s * ei;
                    RE(v, k, q) = s * xr + c * er; IM(v, k, q) = s * xi + c * ei;
                }
                /* rows: new_p = c A_p - s e^{i phi} A_q ; new_q = s A_p + c e^{i phi} A_q */
                for (int k = 0; k < n; ++k) {
                    double xr = RE(a, p, k), xi = IM(a, p, k);
                    double yr = RE(a, q, k), yi = IM(a, q, k);
                    double er = ph_r * yr - ph_i * yi;          /* e^{i phi} * y */
                    double ei = ph_r * yi + ph_i * yr;
                    RE(a, p, k) = c * xr - s * er; IM(a, p, k) = c * xi - s * ei;
                    RE(a, q, k) = s * xr + c * er; IM(a, q, k) = s * xi + c * ei;
                }
                RE(a, p, p) = ap - t * babs; IM(a, p, p) = 0.0;
                RE(a, q, q) = dq + t * babs; IM(a, q, q) = 0.0;
                RE(a, p, q) = IM(a, p, q) = RE(a, q, p) = IM(a, q, p) = 0.0;
            }
        }
    }
    if (!done && offdiag2(n, a) <= tol * tol * fro2) done = 1;
    for (int i = 0; i < n; ++i) w[i] = RE(a, i, i);
    /* selection sort, ascending, moving eigenvector columns along */
    for (int i = 0; i < n - 1; ++i) {
        int k = i;
        for (int j = i + 1; j < n; ++j) if (w[j] < w[k]) k = j;
        if (k != i) {
            double tw = w[i]; w[i] = w[k]; w[k] = tw;
            for (int r = 0; r < n; ++r) {
                double tr = RE(v, r, i), ti = IM(v, r, i);
                RE(v, r, i) = RE(v, r, k); IM(v, r, i) = IM(v, r, k);
                RE(v, r, k) = tr; IM(v, r, k) = ti;
            }
        }
    }
    return done ? sweep : -1;
}
