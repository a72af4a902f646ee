/*
 * nx_oracle.c -- plain FP64 CPU reference for the direct kinematic scattering sum.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file: it exists so that tests, the smoke check and the CPU-baseline leg of
 * the benchmark can check the GPU library against an obviously correct, slow
 * definition.  It shares no code, header or constant with the GPU library.
 *
 * Source: Favre-Nicolin, Coraux, Richard & Renevier, "Fast computing of scattering
 * maps of nanostructures using graphical processing units" (J. Appl. Cryst., 2010).
 *
 *   forward  -- Section 2.1, Eq. 2: A(S) = sum_j f_j exp(2 i pi S.r_j)
 *   loss     -- least-squares intensity misfit L = sum_k (|A_k|^2 - I_k)^2 and its
 *               complex seed G_k = dL/dRe A_k + i dL/dIm A_k.  The paper defines no
 *               loss; this is the fitting objective for strain/displacement fields
 *               that the paper's conclusion (Section 6) motivates.  Parity for the
 *               loss is pinned by a worked value and by finite differences.
 *   adjoint  -- chain rule through Eq. 2:
 *               dL/dr_j = Re sum_k conj(G_k) f_j (2 i pi S_k) exp(2 i pi S_k.r_j)
 *   adjoint_f -- the same chain rule for the factors (A is linear in f_j):
 *               dL/dRe f_j + i dL/dIm f_j = conj( sum_k conj(G_k) exp(2 i pi S_k.r_j) )
 *
 * Conventions (readings of the paper):
 *   - sign +2 i pi as printed in Eq. 2; S in reciprocal-lattice units and r in
 *     lattice (fractional) units, so S.r is in cycles (Section 4.2 converts
 *     orthonormal coordinates to fractional ones before the sum);
 *   - f_j is a constant complex weight per atom (occupancy and species factors
 *     folded in; Section 3 lists (x,y,z,occ) inputs, Section 4.2 factors the
 *     S-dependent atomic factor out of the sum); f == NULL means f_j = 1, the
 *     unit-occupancy sum that the paper's pynx.gpu module evaluates (Section 3);
 *   - the phase is reduced modulo one cycle before cos/sin; exp(2 i pi x) has period
 *     one in x, so this is an identity that only removes libm's own reduction of a
 *     large argument.
 *
 * Arithmetic: IEEE double, no fused multiply-add contraction (-ffp-contract=off),
 * summation in index order.  OpenMP parallelises over independent outputs only;
 * each output's sum is serial and in index order, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* exp(2 i pi phase) with the phase given in cycles (Eq. 2). */
static void cis_cycles(double phase, double *c, double *s)
{
    double t = phase - nearbyint(phase);          /* t in [-1/2, 1/2], exact */
    double a = 2.0 * M_PI * t;
    *c = cos(a);
    *s = sin(a);
}

/* Eq. 2 at every point k: A_k = sum_j f_j exp(2 i pi S_k . r_j).
 * xyz: n_atoms x 3 (row-major), f: n_atoms complex (re, im) or NULL,
 * S: n_points x 3, A: n_points complex (re, im), overwritten. */
void nxo_forward(int64_t n_atoms, const double *xyz, const double *f,
                 int64_t n_points, const double *S, double *A)
{
    int64_t k;
#pragma omp parallel for schedule(dynamic, 16)
    for (k = 0; k < n_points; ++k) {
        const double sx = S[3 * k], sy = S[3 * k + 1], sz = S[3 * k + 2];
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < n_atoms; ++j) {
            double phase = sx * xyz[3 * j] + sy * xyz[3 * j + 1] + sz * xyz[3 * j + 2];
            double c, s;
            cis_cycles(phase, &c, &s);
            double fr = f ? f[2 * j] : 1.0;
            double fi = f ? f[2 * j + 1] : 0.0;
            re += fr * c - fi * s;               /* Re(f_j e^{i theta}) */
            im += fr * s + fi * c;               /* Im(f_j e^{i theta}) */
        }
        A[2 * k] = re;
        A[2 * k + 1] = im;
    }
}

/* Intensity misfit: e_k = |A_k|^2 - I_k, L = sum_k e_k^2 (index order),
 * G_k = dL/dRe A_k + i dL/dIm A_k = 4 e_k A_k.  Returns L. */
double nxo_loss(int64_t n_points, const double *A, const double *I, double *G)
{
    double L = 0.0;
    for (int64_t k = 0; k < n_points; ++k) {
        double re = A[2 * k], im = A[2 * k + 1];
        double e = re * re + im * im - I[k];
        L += e * e;
        if (G) {
            G[2 * k] = 4.0 * e * re;
            G[2 * k + 1] = 4.0 * e * im;
        }
    }
    return L;
}

/* Adjoint of Eq. 2 for a real loss with seed G:
 * grad_j = Re sum_k conj(G_k) * f_j * (2 i pi S_k) * exp(2 i pi S_k . r_j)
 * written term by term: z = conj(G_k) f_j (2 i pi) e^{i theta}, grad_j += Re(z) S_k.
 * grad: n_atoms x 3, overwritten. */
void nxo_adjoint(int64_t n_atoms, const double *xyz, const double *f,
                 int64_t n_points, const double *S, const double *G, double *grad)
{
    int64_t j;
#pragma omp parallel for schedule(dynamic, 4)
    for (j = 0; j < n_atoms; ++j) {
        const double x = xyz[3 * j], y = xyz[3 * j + 1], z = xyz[3 * j + 2];
        const double fr = f ? f[2 * j] : 1.0;
        const double fi = f ? f[2 * j + 1] : 0.0;
        double gx = 0.0, gy = 0.0, gz = 0.0;
        for (int64_t k = 0; k < n_points; ++k) {
            const double sx = S[3 * k], sy = S[3 * k + 1], sz = S[3 * k + 2];
            double c, s;
            cis_cycles(sx * x + sy * y + sz * z, &c, &s);
            /* conj(G_k) * f_j */
            double gr = G[2 * k], gi = -G[2 * k + 1];
            double pr = gr * fr - gi * fi;
            double pi_ = gr * fi + gi * fr;
            /* times 2 i pi */
            double qr = -2.0 * M_PI * pi_;
            double qi = 2.0 * M_PI * pr;
            /* times e^{i theta}; only the real part is needed */
            double zr = qr * c - qi * s;
            gx += zr * sx;
            gy += zr * sy;
            gz += zr * sz;
        }
        grad[3 * j] = gx;
        grad[3 * j + 1] = gy;
        grad[3 * j + 2] = gz;
    }
}

/* Gradient with respect to the per-atom factors: with dA_k = exp(2 i pi S_k.r_j) df_j,
 * dL = Re sum_k conj(G_k) dA_k = Re(W_j df_j), W_j = sum_k conj(G_k) exp(2 i pi S_k.r_j),
 * so dL/dRe f_j = Re W_j and dL/dIm f_j = -Im W_j.  gradf: n_atoms complex, overwritten. */
void nxo_adjoint_f(int64_t n_atoms, const double *xyz, int64_t n_points, const double *S,
                   const double *G, double *gradf)
{
    int64_t j;
#pragma omp parallel for schedule(dynamic, 4)
    for (j = 0; j < n_atoms; ++j) {
        const double x = xyz[3 * j], y = xyz[3 * j + 1], z = xyz[3 * j + 2];
        double wr = 0.0, wi = 0.0;
        for (int64_t k = 0; k < n_points; ++k) {
            double c, s;
            cis_cycles(S[3 * k] * x + S[3 * k + 1] * y + S[3 * k + 2] * z, &c, &s);
            double gr = G[2 * k], gi = -G[2 * k + 1];      /* conj(G_k) */
            wr += gr * c - gi * s;
            wi += gr * s + gi * c;
        }
        gradf[2 * j] = wr;
        gradf[2 * j + 1] = -wi;
    }
}

/* Number of OpenMP threads a parallel region uses (reported by the CPU baseline). */
int nxo_threads(void)
{
    int n = 1;
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
#endif
    return n;
}
