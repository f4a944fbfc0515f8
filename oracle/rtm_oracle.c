/*
 * rtm_oracle.c -- plain FP64 reference of the acoustic RTM time step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or calls this file;
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg load it.  It shares
 * no code, header, table or constant with the HIP path.
 *
 * What it computes (the paper, section II "Structure of the Application": a PDE solver that
 * applies a high-order stencil to a 3-D block of pressure data once per time step):
 *
 *   3-D isotropic acoustic wave equation   (1/v^2) p_tt - lap(p) = f(t) delta(x - x_s),
 *   radius-R star stencil in space (R = 4: 8th order, R = 2: 4th order) with Taylor weights
 *   obtained by Fornberg's recursion (Fornberg 1988), second-order leapfrog in time, and a
 *   Cerjan (1985) sponge that damps both time levels:
 *
 *       L u      = sum over the three axes of [ c0 u + sum_{m=1..R} c_m (u(+m) + u(-m)) ]
 *       u^{n+1}  = g * ( 2 u^n - g * u^{n-1} + kappa * L u^n ),   kappa = (v dt / h)^2.
 *
 * Layout: unpadded arrays, element (i, j, k) at ((k * ny) + j) * nx + i, x fastest.  A neighbour
 * outside the box reads 0 (Dirichlet) or, in periodic mode, the wrapped owned value.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp (no fast-math).  The optional OpenMP loop over z only
 * splits independent point updates between threads, so every thread count gives the same bits.
 */
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_MAX_RADIUS 8

/* ------------------------------------------------------------------------------------------ */
/* Fornberg's recursion for finite-difference weights.                                          */
/*                                                                                              */
/* For nodes x_0..x_{n-1} and an evaluation point z, delta[d][j] is the weight of node j in the  */
/* approximation of the d-th derivative at z that uses all n nodes.  Nodes are added one at a   */
/* time; each new node updates the weights of the old nodes and creates its own.                */
/* ------------------------------------------------------------------------------------------ */
static void fornberg(int n, const double *x, double z, int max_order, double *delta /* [(max_order+1)*n] */)
{
    memset(delta, 0, sizeof(double) * (size_t)(max_order + 1) * (size_t)n);
    double prod_prev = 1.0;             /* product of (x_new - x_old) for the previous new node */
    delta[0 * n + 0] = 1.0;
    for (int i = 1; i < n; ++i) {
        int top = i < max_order ? i : max_order;
        double prod = 1.0;
        double dz_prev = x[i - 1] - z;
        double dz_new = x[i] - z;
        for (int j = 0; j < i; ++j) {
            double gap = x[i] - x[j];
            prod *= gap;
            if (j == i - 1) {
                /* weights of the new node i, built from the last old node's column */
                for (int d = top; d >= 1; --d)
                    delta[d * n + i] = prod_prev * (d * delta[(d - 1) * n + i - 1] - dz_prev * delta[d * n + i - 1]) / prod;
                delta[0 * n + i] = -prod_prev * dz_prev * delta[0 * n + i - 1] / prod;
            }
            /* old node j: correct its weights for the new node */
            for (int d = top; d >= 1; --d)
                delta[d * n + j] = (dz_new * delta[d * n + j] - d * delta[(d - 1) * n + j]) / gap;
            delta[0 * n + j] = dz_new * delta[0 * n + j] / gap;
        }
        prod_prev = prod;
    }
}

/* Second-derivative weights of the centred (2R+1)-point stencil on unit spacing.
 * c[m] = weight of offsets +m and -m, m = 0..R.  Returns 0, or -1 for an unsupported radius. */
int oracle_fd_coefficients(int radius, double *c)
{
    if (radius < 1 || radius > ORACLE_MAX_RADIUS || c == NULL)
        return -1;
    int n = 2 * radius + 1;
    double x[2 * ORACLE_MAX_RADIUS + 1];
    double delta[3 * (2 * ORACLE_MAX_RADIUS + 1)];
    for (int j = 0; j < n; ++j)
        x[j] = (double)(j - radius);           /* nodes -R..R */
    fornberg(n, x, 0.0, 2, delta);
    for (int m = 0; m <= radius; ++m)
        c[m] = delta[2 * n + (radius + m)];
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* Grid access with the boundary rule.                                                         */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int nx, ny, nz;
    int periodic;
} box_t;

static inline double fetch(const box_t *b, const double *u, int i, int j, int k)
{
    if (b->periodic) {
        i = ((i % b->nx) + b->nx) % b->nx;
        j = ((j % b->ny) + b->ny) % b->ny;
        k = ((k % b->nz) + b->nz) % b->nz;
    } else if (i < 0 || i >= b->nx || j < 0 || j >= b->ny || k < 0 || k >= b->nz) {
        return 0.0;
    }
    return u[((size_t)k * b->ny + j) * b->nx + i];
}

/* Dimensionless Laplacian at one point: sum over the axes of c0 u + sum_m c_m (u(+m) + u(-m)). */
static inline double lap_at(const box_t *b, const double *u, const double *c, int radius, int i, int j, int k)
{
    double centre = fetch(b, u, i, j, k);
    double sx = c[0] * centre, sy = c[0] * centre, sz = c[0] * centre;
    for (int m = 1; m <= radius; ++m) {
        sx += c[m] * (fetch(b, u, i + m, j, k) + fetch(b, u, i - m, j, k));
        sy += c[m] * (fetch(b, u, i, j + m, k) + fetch(b, u, i, j - m, k));
        sz += c[m] * (fetch(b, u, i, j, k + m) + fetch(b, u, i, j, k - m));
    }
    return sx + sy + sz;
}

static int set_threads(int nthreads)
{
#ifdef _OPENMP
    return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}

/* out = L u over the whole box. */
void oracle_laplacian(int nx, int ny, int nz, int radius, int periodic, const double *c,
                      const double *u, double *out, int nthreads)
{
    box_t b = {nx, ny, nz, periodic};
    int nt = set_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic) num_threads(nt)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                out[((size_t)k * ny + j) * nx + i] = lap_at(&b, u, c, radius, i, j, k);
}

/* One leapfrog step with sponge:  u_nxt = g (2 u_cur - g u_prv + kappa L u_cur),
 * g = gx[i] gy[j] gz[k].  u_nxt must not alias u_cur; it may alias u_prv. */
void oracle_step(int nx, int ny, int nz, int radius, int periodic, const double *c,
                 const double *kappa, const double *gx, const double *gy, const double *gz,
                 const double *u_cur, const double *u_prv, double *u_nxt, int nthreads)
{
    box_t b = {nx, ny, nz, periodic};
    int nt = set_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic) num_threads(nt)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t p = ((size_t)k * ny + j) * nx + i;
                double g = gx[i] * gy[j] * gz[k];
                double lap = lap_at(&b, u_cur, c, radius, i, j, k);
                u_nxt[p] = g * (2.0 * u_cur[p] - g * u_prv[p] + kappa[p] * lap);
            }
}

/* One step of the transposed recursion (the exact discrete adjoint of oracle_step with the same
 * kappa and sponge).  Writing the forward step as u^{n+1} = A u^n - G^2 u^{n-1} with
 * A = G (2I + K L), G = diag(g), K = diag(kappa), and L symmetric, its transpose is
 * A^T = (2I + L K) G, so the adjoint state runs backwards as
 *
 *       mu_out = 2 g mu_a + L(kappa g mu_a) - g^2 mu_b,
 *
 * where mu_a is the adjoint state one level later and mu_b two levels later.  The scratch array
 * `tmp` (size nx*ny*nz) holds kappa g mu_a.  mu_out may alias mu_b. */
void oracle_adjoint_step(int nx, int ny, int nz, int radius, int periodic, const double *c,
                         const double *kappa, const double *gx, const double *gy, const double *gz,
                         const double *mu_a, const double *mu_b, double *mu_out, double *tmp, int nthreads)
{
    box_t b = {nx, ny, nz, periodic};
    int nt = set_threads(nthreads);
    (void)nt;
#pragma omp parallel for schedule(dynamic) num_threads(nt)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t p = ((size_t)k * ny + j) * nx + i;
                tmp[p] = kappa[p] * (gx[i] * gy[j] * gz[k]) * mu_a[p];
            }
#pragma omp parallel for schedule(dynamic) num_threads(nt)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t p = ((size_t)k * ny + j) * nx + i;
                double g = gx[i] * gy[j] * gz[k];
                double lap = lap_at(&b, tmp, c, radius, i, j, k);
                mu_out[p] = 2.0 * g * mu_a[p] + lap - g * g * mu_b[p];
            }
}

int oracle_abi_version(void) { return 1; }
