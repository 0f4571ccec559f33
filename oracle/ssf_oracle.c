/*
 * ssf_oracle.c -- plain, slow FP64 CPU oracle for the Fourier split-operator
 * propagation of the three-dimensional time-dependent Schroedinger equation
 * (hbar = m = 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; the product path
 * never links or calls it.
 *
 * Source of the method: T. Morgan, L. J. O'Riordan, N. Crowley, B. O'Sullivan,
 * Th. Busch, "Coherent transport by adiabatic passage on atom chips",
 * arXiv:1309.2451.
 *   - Sec. IV (MPI and CUDA), first paragraph: the time-dependent Schroedinger
 *     equation is integrated with the Fourier split-operator method; every time
 *     step is a handful of 3D Fourier transforms and pointwise complex
 *     multiplications by exponentials of the potential and kinetic operators.
 *   - Sec. IV, second paragraph: the momentum grid is bounded by
 *     p_max = pi N / L (L the box length along that axis).
 *   - Sec. V, second paragraph: the initial transverse state is the
 *     numerically determined ground state (here: imaginary-time propagation).
 *   - Sec. V (Fig. 4, Fig. 6): the observable is the population found in each
 *     of the three waveguides; the final population in the target guide is the
 *     transfer fidelity.
 * Readings of points the paper leaves open (splitting order V/2-T-V/2, FFT
 * sign and normalisation, periodic box with the upper end excluded, guide
 * regions as fixed x partitions, the Gaussian waveguide potential standing in
 * for the chip's magnetic one) are listed in the design notes of the
 * repository, each with its reason.
 *
 * Conventions (all FP64):
 *   grid: x_i = lo + i*(hi-lo)/n, i = 0..n-1 (periodic, hi excluded); arrays
 *         are (nz, ny, nx) with x fastest; complex values are interleaved
 *         (re, im) pairs of doubles.
 *   FFT:  forward  X[k] = sum_j x[j] exp(-2 pi i j k / n)  (unnormalised),
 *         inverse  x[j] = (1/n) sum_k X[k] exp(+2 pi i j k / n).
 *   k:    k_j = (2 pi / L) * (2j < n ? j : j - n), L = hi - lo.
 *
 * Build: gcc -O2 -std=c99 -fPIC -shared -fopenmp ssf_oracle.c -lm
 * (no -ffast-math, no -march: FP64 results do not depend on the thread count
 * because threads only ever split independent pencils or z-planes.)
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double TWO_PI = 6.283185307179586476925286766559;

/* ------------------------------------------------------------------------ */
/* 1-D DFT by recursive mixed-radix Cooley-Tukey (decimation in time).       */
/* ------------------------------------------------------------------------ */

/* Smallest prime factor of n (n >= 2). */
static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* Table w[t] = exp(sign * 2 pi i t / n0), t = 0..n0-1, each entry from its own
 * cos/sin call (no recurrence). */
static cplx *twiddle_table(int n0, int sign)
{
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)n0);
    for (int t = 0; t < n0; ++t) {
        double a = TWO_PI * (double)t / (double)n0;
        w[t] = cos(a) + (double)sign * sin(a) * I;
    }
    return w;
}

/*
 * out[0..n-1] = DFT_n of in[0], in[is], in[2 is], ...  with kernel
 * exp(sign 2 pi i j k / n).  n divides n0 and w is the n0-table.
 * Split n = p*m with p the smallest prime factor:
 *   X[k1 + m k2] = sum_{q<p} w_n^{q (k1 + m k2)} Y_q[k1],
 *   Y_q = DFT_m of the subsequence in[q], in[q+p], ...
 */
static void dft_rec(int n, const cplx *in, ptrdiff_t is, cplx *out,
                    const cplx *w, int n0)
{
    if (n == 1) { out[0] = in[0]; return; }
    int p = smallest_factor(n);
    int m = n / p;
    for (int q = 0; q < p; ++q)
        dft_rec(m, in + (ptrdiff_t)q * is, is * p, out + (size_t)q * m, w, n0);
    int stride = n0 / n;                  /* w_n^t = w[t * n0/n] */
    cplx *t = (cplx *)malloc(sizeof(cplx) * (size_t)p);
    for (int k1 = 0; k1 < m; ++k1) {
        for (int q = 0; q < p; ++q) t[q] = out[(size_t)q * m + k1];
        for (int k2 = 0; k2 < p; ++k2) {
            int k = k1 + m * k2;
            cplx s = 0.0;
            for (int q = 0; q < p; ++q) {
                long e = ((long)q * (long)k) % n;
                s += w[e * stride] * t[q];
            }
            out[k] = s;
        }
    }
    free(t);
}

/* In-place 1-D transform of n interleaved complex values, unnormalised,
 * kernel exp(sign 2 pi i j k / n). */
void orc_fft1d(double *data, int n, int sign)
{
    if (n <= 1) return;
    cplx *in = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *w = twiddle_table(n, sign);
    for (int j = 0; j < n; ++j) in[j] = data[2 * j] + data[2 * j + 1] * I;
    dft_rec(n, in, 1, out, w, n);
    for (int j = 0; j < n; ++j) { data[2 * j] = creal(out[j]); data[2 * j + 1] = cimag(out[j]); }
    free(in); free(out); free(w);
}

/* Apply the 1-D transform to every pencil along one axis of a (nz,ny,nx)
 * complex array.  axis 0 = x, 1 = y, 2 = z. */
static void fft_axis(cplx *psi, int nx, int ny, int nz, int axis, int sign)
{
    int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
    if (n <= 1) return;
    ptrdiff_t stride = axis == 0 ? 1 : (axis == 1 ? nx : (ptrdiff_t)nx * ny);
    long npencil = (long)nx * ny * nz / n;
    cplx *w = twiddle_table(n, sign);
    #pragma omp parallel
    {
        cplx *in = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        cplx *out = (cplx *)malloc(sizeof(cplx) * (size_t)n);
        #pragma omp for schedule(static)
        for (long pc = 0; pc < npencil; ++pc) {
            ptrdiff_t base;
            if (axis == 0) base = (ptrdiff_t)pc * nx;
            else if (axis == 1) { long x = pc % nx, z = pc / nx; base = (ptrdiff_t)z * nx * ny + x; }
            else base = (ptrdiff_t)pc;      /* pc = y*nx + x */
            for (int j = 0; j < n; ++j) in[j] = psi[base + (ptrdiff_t)j * stride];
            dft_rec(n, in, 1, out, w, n);
            for (int j = 0; j < n; ++j) psi[base + (ptrdiff_t)j * stride] = out[j];
        }
        free(in); free(out);
    }
    free(w);
}

/* 3-D transform: 1-D transforms along x, then y, then z.  dir = -1 forward
 * (unnormalised), dir = +1 inverse (scaled by 1/(nx ny nz)). */
static void fft3d(cplx *psi, int nx, int ny, int nz, int dir)
{
    fft_axis(psi, nx, ny, nz, 0, dir);
    fft_axis(psi, nx, ny, nz, 1, dir);
    fft_axis(psi, nx, ny, nz, 2, dir);
    if (dir > 0) {
        double s = 1.0 / ((double)nx * ny * nz);
        long tot = (long)nx * ny * nz;
        for (long i = 0; i < tot; ++i) psi[i] *= s;
    }
}

void orc_fft3d(double *psi, int nx, int ny, int nz, int dir)
{
    fft3d((cplx *)psi, nx, ny, nz, dir);
}

/* Apply the 1-D transform along one axis only (unnormalised, kernel sign). */
void orc_fft_axis(double *psi, int nx, int ny, int nz, int axis, int sign)
{
    fft_axis((cplx *)psi, nx, ny, nz, axis, sign);
}

/* ------------------------------------------------------------------------ */
/* Grids.                                                                    */
/* ------------------------------------------------------------------------ */

typedef struct { int n[3]; double lo[3], hi[3]; } grid_t;

static grid_t make_grid(const int *n, const double *lo, const double *hi)
{
    grid_t g;
    for (int a = 0; a < 3; ++a) { g.n[a] = n[a]; g.lo[a] = lo[a]; g.hi[a] = hi[a]; }
    return g;
}

static double grid_step(const grid_t *g, int a) { return (g->hi[a] - g->lo[a]) / g->n[a]; }
static double grid_coord(const grid_t *g, int a, int i) { return g->lo[a] + i * grid_step(g, a); }
static double grid_dv(const grid_t *g) { return grid_step(g, 0) * grid_step(g, 1) * grid_step(g, 2); }
static long grid_points(const grid_t *g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

/* Angular wavenumber of FFT bin j on an axis of n points and length L
 * (Sec. IV: |k| <= pi n / L). */
static double wavenumber(int j, int n, double L)
{
    int m = (2 * j < n) ? j : j - n;      /* bins above n/2 are negative */
    return TWO_PI / L * (double)m;
}

void orc_kgrid(int n, double L, double *k)
{
    for (int j = 0; j < n; ++j) k[j] = wavenumber(j, n, L);
}

/* ------------------------------------------------------------------------ */
/* One Strang step V/2 - T - V/2 of the Fourier split-operator method.       */
/* ------------------------------------------------------------------------ */

/* psi <- exp(-i V dt/2) psi (real time) or exp(-V dt/2) psi (imaginary). */
static void potential_half(cplx *psi, const double *V, long tot, double dt, int imag)
{
    if (!V) return;
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < tot; ++i) {
        double a = V[i] * dt * 0.5;
        cplx f = imag ? exp(-a) : (cos(a) - sin(a) * I);
        psi[i] *= f;
    }
}

/* psi_hat <- exp(-i k^2 dt/2) psi_hat (real) or exp(-k^2 dt/2) psi_hat. */
static void kinetic_full(cplx *psih, const grid_t *g, double dt, int imag)
{
    int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    double Lx = g->hi[0] - g->lo[0], Ly = g->hi[1] - g->lo[1], Lz = g->hi[2] - g->lo[2];
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        double kz = wavenumber(z, nz, Lz);
        for (int y = 0; y < ny; ++y) {
            double ky = wavenumber(y, ny, Ly);
            for (int x = 0; x < nx; ++x) {
                double kx = wavenumber(x, nx, Lx);
                double a = (kx * kx + ky * ky + kz * kz) * dt * 0.5;
                cplx f = imag ? exp(-a) : (cos(a) - sin(a) * I);
                psih[((long)z * ny + y) * nx + x] *= f;
            }
        }
    }
}

/*
 * Sums over the grid.  The observables are plain sums over every grid point
 * (Sec. V: the population of a guide is the probability summed over its
 * region); a running FP64 sum over the 10^7 - 10^8 points of a large grid
 * carries a rounding error of order 1e-13 relative (one rounding per term),
 * so every sum over the grid uses Neumaier's compensated summation, whose
 * result lies within a few units in the last place of the exact sum: the
 * running sum s and, in c, the rounding error of every addition.
 */
typedef struct { double s, c; } ksum_t;

static void ksum_add(ksum_t *k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}

static double ksum_value(const ksum_t *k) { return k->s + k->c; }

static double sum_abs2(const cplx *psi, long tot)
{
    ksum_t s = {0.0, 0.0};
    for (long i = 0; i < tot; ++i) ksum_add(&s, creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]));
    return ksum_value(&s);
}

static void one_step(cplx *psi, const double *V, const grid_t *g, double dt, int imag)
{
    long tot = grid_points(g);
    potential_half(psi, V, tot, dt, imag);
    fft3d(psi, g->n[0], g->n[1], g->n[2], -1);
    kinetic_full(psi, g, dt, imag);
    fft3d(psi, g->n[0], g->n[1], g->n[2], +1);
    potential_half(psi, V, tot, dt, imag);
}

/*
 * The other symmetric ordering, T/2 - V - T/2 (Sec. IV counts four Fourier
 * transforms and three multiplications per step, which is this form taken
 * step by step): half a kinetic step in momentum space, the full potential
 * phase in position space, half a kinetic step again.
 */
static void one_step_tvt(cplx *psi, const double *V, const grid_t *g, double dt, int imag)
{
    long tot = grid_points(g);
    fft3d(psi, g->n[0], g->n[1], g->n[2], -1);
    kinetic_full(psi, g, 0.5 * dt, imag);
    fft3d(psi, g->n[0], g->n[1], g->n[2], +1);
    potential_half(psi, V, tot, 2.0 * dt, imag);
    fft3d(psi, g->n[0], g->n[1], g->n[2], -1);
    kinetic_full(psi, g, 0.5 * dt, imag);
    fft3d(psi, g->n[0], g->n[1], g->n[2], +1);
}

/*
 * nsteps Strang steps, order 0 = V/2 - T - V/2, 1 = T/2 - V - T/2.
 * Real time (imag = 0): no renormalisation.
 * Imaginary time (imag = 1): after every step psi is rescaled to
 * sum |psi|^2 dV = 1 and, if edecay != NULL, edecay[s] receives
 * -ln(||psi_{s+1}|| / ||psi_s||) / dt measured before the rescale (the
 * input is taken as it is, so edecay[0] assumes a normalised input).
 * V may be NULL (free particle).
 */
void orc_step_order(double *psi_, const double *V, const int *n, const double *lo, const double *hi,
                    double dt, long nsteps, int imag, double *edecay, int order)
{
    grid_t g = make_grid(n, lo, hi);
    cplx *psi = (cplx *)psi_;
    long tot = grid_points(&g);
    double dv = grid_dv(&g);
    double prev = sqrt(sum_abs2(psi, tot) * dv);
    for (long s = 0; s < nsteps; ++s) {
        if (order == 1) one_step_tvt(psi, V, &g, dt, imag);
        else one_step(psi, V, &g, dt, imag);
        if (imag) {
            double nrm = sqrt(sum_abs2(psi, tot) * dv);
            if (edecay) edecay[s] = -log(nrm / prev) / dt;
            double inv = 1.0 / nrm;
            for (long i = 0; i < tot; ++i) psi[i] *= inv;
            prev = 1.0;
        }
    }
}

void orc_step(double *psi_, const double *V, const int *n, const double *lo, const double *hi,
              double dt, long nsteps, int imag, double *edecay)
{
    orc_step_order(psi_, V, n, lo, hi, dt, nsteps, imag, edecay, 0);
}

/* ------------------------------------------------------------------------ */
/* Observables (Sec. V: populations of the three guides).                    */
/* ------------------------------------------------------------------------ */

/*
 * out[0] = sum |psi|^2 dV                       (norm)
 * out[1..3] = sum x|psi|^2 dV, sum y|psi|^2 dV, sum z|psi|^2 dV
 * out[4] = P1 = sum over x < x_lo, out[5] = P2 = sum over x_lo <= x <= x_hi,
 * out[6] = P3 = sum over x > x_hi              (guide populations)
 * out[7] = <H> = sum (k^2/2)|psi_hat|^2 dV / N + sum V |psi|^2 dV
 *          (psi_hat the unnormalised forward FFT; V may be NULL -> 0).
 */
void orc_observables(const double *psi_, const double *V, const int *n, const double *lo,
                     const double *hi, double x_lo, double x_hi, double *out)
{
    grid_t g = make_grid(n, lo, hi);
    const cplx *psi = (const cplx *)psi_;
    int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    long tot = grid_points(&g);
    double dv = grid_dv(&g);
    ksum_t s[8];
    for (int q = 0; q < 8; ++q) s[q].s = s[q].c = 0.0;
    for (int z = 0; z < nz; ++z) {
        double zc = grid_coord(&g, 2, z);
        for (int y = 0; y < ny; ++y) {
            double yc = grid_coord(&g, 1, y);
            for (int x = 0; x < nx; ++x) {
                double xc = grid_coord(&g, 0, x);
                long i = ((long)z * ny + y) * nx + x;
                double r = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
                ksum_add(&s[0], r);
                ksum_add(&s[1], xc * r); ksum_add(&s[2], yc * r); ksum_add(&s[3], zc * r);
                if (xc < x_lo) ksum_add(&s[4], r);
                else if (xc > x_hi) ksum_add(&s[6], r);
                else ksum_add(&s[5], r);
                if (V) ksum_add(&s[7], V[i] * r);
            }
        }
    }
    cplx *ph = (cplx *)malloc(sizeof(cplx) * (size_t)tot);
    memcpy(ph, psi, sizeof(cplx) * (size_t)tot);
    fft3d(ph, nx, ny, nz, -1);
    ksum_t kin = {0.0, 0.0};
    double Lx = g.hi[0] - g.lo[0], Ly = g.hi[1] - g.lo[1], Lz = g.hi[2] - g.lo[2];
    for (int z = 0; z < nz; ++z) {
        double kz = wavenumber(z, nz, Lz);
        for (int y = 0; y < ny; ++y) {
            double ky = wavenumber(y, ny, Ly);
            for (int x = 0; x < nx; ++x) {
                double kx = wavenumber(x, nx, Lx);
                long i = ((long)z * ny + y) * nx + x;
                double r = creal(ph[i]) * creal(ph[i]) + cimag(ph[i]) * cimag(ph[i]);
                ksum_add(&kin, 0.5 * (kx * kx + ky * ky + kz * kz) * r);
            }
        }
    }
    free(ph);
    for (int q = 0; q < 7; ++q) out[q] = ksum_value(&s[q]) * dv;
    out[7] = ksum_value(&kin) * dv / (double)tot + ksum_value(&s[7]) * dv;
}

/*
 * Guide populations with plane-dependent boundaries (Sec. V, Fig. 4: the
 * population of each waveguide as the guides move): out[0] = P1 = sum over
 * x < x_lo[z], out[2] = P3 = sum over x > x_hi[z], out[1] = P2 the rest,
 * each times dV.
 */
void orc_populations_z(const double *psi_, const int *n, const double *lo, const double *hi,
                       const double *x_lo, const double *x_hi, double *out)
{
    grid_t g = make_grid(n, lo, hi);
    const cplx *psi = (const cplx *)psi_;
    int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    double dv = grid_dv(&g);
    ksum_t p[3] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                double xc = grid_coord(&g, 0, x);
                long i = ((long)z * ny + y) * nx + x;
                double r = creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
                if (xc < x_lo[z]) ksum_add(&p[0], r);
                else if (xc > x_hi[z]) ksum_add(&p[2], r);
                else ksum_add(&p[1], r);
            }
    for (int q = 0; q < 3; ++q) out[q] = ksum_value(&p[q]) * dv;
}

/*
 * Density in the x-z plane integrated over y (Sec. V, Fig. 5):
 * out[z * nx + x] = sum_y |psi(x, y, z)|^2 dy.
 */
void orc_density_xz(const double *psi_, const int *n, const double *lo, const double *hi, double *out)
{
    grid_t g = make_grid(n, lo, hi);
    const cplx *psi = (const cplx *)psi_;
    int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    double dy = (g.hi[1] - g.lo[1]) / ny;
    for (int z = 0; z < nz; ++z)
        for (int x = 0; x < nx; ++x) {
            double s = 0.0;
            for (int y = 0; y < ny; ++y) {
                long i = ((long)z * ny + y) * nx + x;
                s += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
            }
            out[(long)z * nx + x] = s * dy;
        }
}

/* ------------------------------------------------------------------------ */
/* Three-guide potential (Gaussian stand-in for the chip's waveguides).      */
/* ------------------------------------------------------------------------ */

/*
 * V(x,y,z) = - sum_j v0[j] exp(-((x - xc[j][z])^2 + y^2) / (2 sigma[j]^2)),
 * xc is (nguides, nz): the centre of guide j in the plane z.
 */
void orc_ctap_potential(double *V, const int *n, const double *lo, const double *hi,
                        int nguides, const double *v0, const double *sigma, const double *xc)
{
    grid_t g = make_grid(n, lo, hi);
    int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            double yc = grid_coord(&g, 1, y);
            for (int x = 0; x < nx; ++x) {
                double xp = grid_coord(&g, 0, x);
                double v = 0.0;
                for (int j = 0; j < nguides; ++j) {
                    double d = xp - xc[(long)j * nz + z];
                    v -= v0[j] * exp(-(d * d + yc * yc) / (2.0 * sigma[j] * sigma[j]));
                }
                V[((long)z * ny + y) * nx + x] = v;
            }
        }
}

/* ------------------------------------------------------------------------ */
/* Atom-chip potential: thin current-carrying wires on the chip surface plus  */
/* homogeneous bias and offset fields (Sec. III) and the longitudinal         */
/* harmonic trap V_z (Sec. III, last paragraphs).                             */
/* ------------------------------------------------------------------------ */

/*
 * Magnetic field (tesla) of the wires alone at point (px, py, pz).  Lengths
 * are in units of length_unit metres.  Wire w is the polyline through the
 * points (path[2k], 0, path[2k+1]) (x and z; the wires lie in the chip plane
 * y = 0) carrying current[w] amperes from its first point to its last.
 *
 * Biot-Savart law (Sec. III) for one straight segment from A to B, written
 * out: with L = B - A, a = P - A, b = P - B, the line integral of
 * dl x r_hat / r^2 over the segment equals
 *     (L x a) / |L x a|^2 * (L.a / |a| - L.b / |b|),
 * the classic finite-wire result (mu0 I / (4 pi rho)) (cos t1 - cos t2) along
 * the azimuthal direction, with rho = |L x a| / |L| the distance from the
 * segment's line.  Points on that line get no contribution from it.
 */
static void wire_field(double px, double py, double pz, int nwires, const int *npts,
                       const double *path, const double *current, double length_unit, double *B)
{
    const double mu0_4pi = 1.25663706212e-6 / (4.0 * 3.14159265358979323846);
    double bx = 0.0, by = 0.0, bz = 0.0;
    const double *pp = path;
    for (int w = 0; w < nwires; ++w) {
        double k = mu0_4pi * current[w] / length_unit;
        for (int s = 0; s + 1 < npts[w]; ++s) {
            double Ax = pp[2 * s], Az = pp[2 * s + 1];
            double Bx = pp[2 * s + 2], Bz = pp[2 * s + 3];
            double Lx = Bx - Ax, Ly = 0.0, Lz = Bz - Az;
            double ax = px - Ax, ay = py, az = pz - Az;
            double bxv = px - Bx, byv = py, bzv = pz - Bz;
            /* c = L x a */
            double cx = Ly * az - Lz * ay;
            double cy = Lz * ax - Lx * az;
            double cz = Lx * ay - Ly * ax;
            double c2 = cx * cx + cy * cy + cz * cz;
            if (c2 == 0.0)
                continue;
            double la = (Lx * ax + Ly * ay + Lz * az) / sqrt(ax * ax + ay * ay + az * az);
            double lb = (Lx * bxv + Ly * byv + Lz * bzv) / sqrt(bxv * bxv + byv * byv + bzv * bzv);
            double f = k * (la - lb) / c2;
            bx += f * cx;
            by += f * cy;
            bz += f * cz;
        }
        pp += 2 * npts[w];
    }
    B[0] = bx;
    B[1] = by;
    B[2] = bz;
}

/*
 * The potential from the wires' field Bw at a point:
 *     V = mu_over_e0 (|B| - b_ip) + omega_z^2 (z - z_c)^2 / 2,
 * B = Bw + (b_bias, 0, b_ip), the magnetic energy of a low-field-seeking
 * atom (magnetic moment mu, energy unit E0, so mu_over_e0 = mu / E0 per
 * tesla) measured from its value at a field of magnitude b_ip, plus the
 * longitudinal trap of frequency omega_z (in inverse time units) centred at
 * z_c.  |B| - b_ip is evaluated as (|B|^2 - b_ip^2) / (|B| + b_ip) with
 * |B|^2 - b_ip^2 = Bx^2 + By^2 + Bwz (Bwz + 2 b_ip): the same number without
 * the cancellation of two nearly equal magnitudes at the guide centres.
 */
static double chip_value(const double *Bw, double dz, double b_bias, double b_ip, double mu_over_e0,
                         double omega_z)
{
    double bx = Bw[0] + b_bias, by = Bw[1], bz = Bw[2] + b_ip;
    double mag = sqrt(bx * bx + by * by + bz * bz);
    double excess = (bx * bx + by * by + Bw[2] * (Bw[2] + 2.0 * b_ip)) / (mag + b_ip);
    return mu_over_e0 * excess + 0.5 * omega_z * omega_z * dz * dz;
}

/* V at m points pts[3i..3i+2] = (x, y, z). */
void orc_chip_potential_points(double *V, const double *pts, long m, int nwires, const int *npts,
                               const double *path, const double *current, double b_bias, double b_ip,
                               double length_unit, double mu_over_e0, double omega_z, double z_c)
{
    #pragma omp parallel for schedule(static)
    for (long i = 0; i < m; ++i) {
        double Bw[3];
        wire_field(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2], nwires, npts, path, current, length_unit, Bw);
        V[i] = chip_value(Bw, pts[3 * i + 2] - z_c, b_bias, b_ip, mu_over_e0, omega_z);
    }
}

/* The same potential on the whole grid, (nz, ny, nx). */
void orc_chip_potential(double *V, const int *n, const double *lo, const double *hi, int nwires,
                        const int *npts, const double *path, const double *current, double b_bias,
                        double b_ip, double length_unit, double mu_over_e0, double omega_z, double z_c)
{
    grid_t g = make_grid(n, lo, hi);
    int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        double zc = grid_coord(&g, 2, z);
        for (int y = 0; y < ny; ++y) {
            double yc = grid_coord(&g, 1, y);
            for (int x = 0; x < nx; ++x) {
                double Bw[3];
                wire_field(grid_coord(&g, 0, x), yc, zc, nwires, npts, path, current, length_unit, Bw);
                V[((long)z * ny + y) * nx + x] = chip_value(Bw, zc - z_c, b_bias, b_ip, mu_over_e0, omega_z);
            }
        }
    }
}

/* The total field Bw + (b_bias, 0, b_ip) (tesla) at m points, (m, 3). */
void orc_chip_field_points(double *Bout, const double *pts, long m, int nwires, const int *npts,
                           const double *path, const double *current, double b_bias, double b_ip,
                           double length_unit)
{
    for (long i = 0; i < m; ++i) {
        wire_field(pts[3 * i], pts[3 * i + 1], pts[3 * i + 2], nwires, npts, path, current, length_unit,
                   Bout + 3 * i);
        Bout[3 * i] += b_bias;
        Bout[3 * i + 2] += b_ip;
    }
}

/* ------------------------------------------------------------------------ */
/* Clamped uniform cubic B-splines (guide-centre profile parameterisation).  */
/* ------------------------------------------------------------------------ */

/*
 * B[iz*M + m] = B_m(z[iz]) for M >= 4 cubic B-splines on the clamped knot
 * vector over [a, b]: a four times, a + i (b-a)/(M-3) for i = 1..M-4, b four
 * times.  Cox-de Boor recursion; at z == b the last basis function is 1.
 */
void orc_bspline_basis(int M, double a, double b, const double *z, int nz, double *B)
{
    int nk = M + 4;
    double *t = (double *)malloc(sizeof(double) * (size_t)nk);
    int nseg = M - 3;
    for (int i = 0; i < 4; ++i) { t[i] = a; t[nk - 1 - i] = b; }
    for (int i = 1; i < nseg; ++i) t[3 + i] = a + (b - a) * (double)i / (double)nseg;
    double *N0 = (double *)malloc(sizeof(double) * (size_t)nk);
    for (int iz = 0; iz < nz; ++iz) {
        double u = z[iz];
        /* degree 0 */
        for (int i = 0; i < nk - 1; ++i) {
            N0[i] = (t[i] <= u && u < t[i + 1]) ? 1.0 : 0.0;
        }
        if (u >= b) { for (int i = 0; i < nk - 1; ++i) N0[i] = 0.0; N0[M - 1] = 1.0; }
        /* degrees 1..3 */
        for (int d = 1; d <= 3; ++d) {
            for (int i = 0; i < nk - 1 - d; ++i) {
                double l = 0.0, r = 0.0;
                double dl = t[i + d] - t[i], dr = t[i + d + 1] - t[i + 1];
                if (dl > 0.0) l = (u - t[i]) / dl * N0[i];
                if (dr > 0.0) r = (t[i + d + 1] - u) / dr * N0[i + 1];
                N0[i] = l + r;
            }
        }
        if (u >= b) { for (int m = 0; m < M; ++m) B[(long)iz * M + m] = (m == M - 1) ? 1.0 : 0.0; }
        else for (int m = 0; m < M; ++m) B[(long)iz * M + m] = N0[m];
    }
    free(t); free(N0);
}

/* ------------------------------------------------------------------------ */
/* Adjoint of the final target-guide population.                             */
/* ------------------------------------------------------------------------ */

/* dV/dxc_j at every grid point of plane z: -v0 e_j (x - xc)/sigma^2 with
 * e_j = exp(-((x-xc)^2+y^2)/(2 sigma^2)). */
static double dV_dxc(const grid_t *g, int x, int y, int z, double v0, double sig, double xcz)
{
    double xp = grid_coord(g, 0, x), yc = grid_coord(g, 1, y);
    double d = xp - xcz;
    double e = exp(-(d * d + yc * yc) / (2.0 * sig * sig));
    return -v0 * e * d / (sig * sig);
}

/* G[j][z] += dt * sum_{x,y} dV/dxc_j * Im(conj(lam) * psi) * dV */
static void accumulate_G(double *G, const grid_t *g, const cplx *lam, const cplx *psi,
                         int nguides, const double *v0, const double *sigma, const double *xc,
                         double dt)
{
    int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    double dv = grid_dv(g);
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int j = 0; j < nguides; ++j) {
            double acc = 0.0;
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    long i = ((long)z * ny + y) * nx + x;
                    double im = cimag(conj(lam[i]) * psi[i]);
                    acc += dV_dxc(g, x, y, z, v0[j], sigma[j], xc[(long)j * nz + z]) * im;
                }
            G[(long)j * nz + z] += dt * acc * dv;
        }
}

/*
 * Real-time propagation of psi0 through nsteps Strang steps in the guide
 * potential built from (v0, sigma, xc), then the final population
 * F = sum_{x > x_hi} |psi_N|^2 dV (returned in *F) and its derivative with
 * respect to every guide centre xc[j][z] (written to G, shape (nguides, nz)).
 *
 * Reverse-mode chain rule through every factor of every step, with all forward
 * states stored: with A = exp(-i V dt/2) and B the kinetic factor, a step is
 * psi -> A B A psi.  Each A factor contributes dt * sum dV/dxc Im(conj(lam) u) dV,
 * where u is the state just after that factor and lam the adjoint at the same
 * point; lam is carried backwards through A^dagger and B^dagger.
 * psi_out (optional) receives psi_N.
 */
void orc_adjoint_ctap(const double *psi0_, const int *n, const double *lo, const double *hi,
                      int nguides, const double *v0, const double *sigma, const double *xc,
                      double dt, long nsteps, double x_hi, double *F, double *G, double *psi_out)
{
    grid_t g = make_grid(n, lo, hi);
    long tot = grid_points(&g);
    double dv = grid_dv(&g);
    int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    double *V = (double *)malloc(sizeof(double) * (size_t)tot);
    orc_ctap_potential(V, n, lo, hi, nguides, v0, sigma, xc);

    cplx *states = (cplx *)malloc(sizeof(cplx) * (size_t)tot * (size_t)(nsteps + 1));
    memcpy(states, psi0_, sizeof(cplx) * (size_t)tot);
    for (long s = 0; s < nsteps; ++s) {
        cplx *nxt = states + (size_t)(s + 1) * tot;
        memcpy(nxt, states + (size_t)s * tot, sizeof(cplx) * (size_t)tot);
        one_step(nxt, V, &g, dt, 0);
    }
    cplx *psiN = states + (size_t)nsteps * tot;
    if (psi_out) memcpy(psi_out, psiN, sizeof(cplx) * (size_t)tot);

    /* F and the terminal adjoint lam_N = M psi_N (M the target-region mask). */
    cplx *lam = (cplx *)malloc(sizeof(cplx) * (size_t)tot);
    double f = 0.0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = ((long)z * ny + y) * nx + x;
                int in = grid_coord(&g, 0, x) > x_hi;
                lam[i] = in ? psiN[i] : 0.0;
                if (in) f += creal(psiN[i]) * creal(psiN[i]) + cimag(psiN[i]) * cimag(psiN[i]);
            }
    *F = f * dv;
    memset(G, 0, sizeof(double) * (size_t)nguides * nz);

    cplx *u = (cplx *)malloc(sizeof(cplx) * (size_t)tot);
    for (long s = nsteps - 1; s >= 0; --s) {
        /* second A factor of step s: state just after it is psi_{s+1} */
        accumulate_G(G, &g, lam, states + (size_t)(s + 1) * tot, nguides, v0, sigma, xc, dt);
        potential_half(lam, V, tot, -dt, 0);                 /* A^dagger */
        fft3d(lam, nx, ny, nz, -1);                          /* B^dagger */
        kinetic_full(lam, &g, -dt, 0);
        fft3d(lam, nx, ny, nz, +1);
        /* first A factor of step s: state just after it is A psi_s */
        memcpy(u, states + (size_t)s * tot, sizeof(cplx) * (size_t)tot);
        potential_half(u, V, tot, dt, 0);
        accumulate_G(G, &g, lam, u, nguides, v0, sigma, xc, dt);
        potential_half(lam, V, tot, -dt, 0);                 /* A^dagger */
    }
    free(u); free(lam); free(states); free(V);
}

/* Threads of the parallel loops (over independent pencils and planes: the
 * results do not depend on the count). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0)
        omp_set_num_threads(n);
#else
    (void)n;
#endif
}
