/*
 * FP64 reference stepper for the generalized FDTD scheme in 2D (TE and TM
 * polarizations, interfaces normal to the velocity).
 *
 * TEST INFRASTRUCTURE.  This file is the oracle for the 2D path: a plain,
 * slow, loop-by-loop statement of what the path computes, used only by the
 * test-suite and the benchmark's CPU leg.  It shares no code, header or
 * table with the HIP library, and the library never calls it.
 *
 * The paper discretizes only the 1D case (Section 4, eq. (10a)-(10d) with
 * Table 1).  Its 3D mixed-field equations (eq. (6)) and constitutive
 * relations (eq. (7)) are read here for fields independent of y, motion
 * v = beta z^ and a moving modulation eps(z - vt), mu(z - vt) whose
 * interfaces are normal to v (the case Section 3 assumes, eq. (3)):
 *   curl (v x F) = v (div F) - (v . grad) F = -v dF/dz   (div B = 0, and
 *   div D = 0 away from sources), so each component obeys
 *   dB/dt = -curl E* - v dB/dz,  dD/dt = curl H* - v dD/dz,
 * with the star fields of eq. (2):
 *   TE (E_y, H_x, H_z):  E*_y = D_y/eps + v B_x,  H*_x = B_x/mu + v D_y,
 *                        H*_z = B_z/mu;
 *   TM (H_y, E_x, E_z):  E*_x = D_x/eps - v B_y,  H*_y = B_y/mu - v D_x,
 *                        E*_z = D_z/eps.
 * The z-derivatives of the velocity terms and the velocity averages take
 * the Table 1 stencils and time levels of the 1D scheme (column a for
 * v >= 0, b for v < 0) on each lattice; the curls are the Yee differences.
 *
 * Grid (square cells, dx = dz = 1, time step S = dt/dz = dt/dx): nx
 * columns, periodic in x; along z, E-lattice nodes k = 0..nz-1 and
 * H-lattice nodes j = 0..nz-2 at j+1/2 (both ends are E-lattice nodes, as
 * in 1D), or nz of each on a z-ring.
 *   TE:  D = D_y at (i, k)        B = B_x at (i, j+1/2)   C = B_z at (i+1/2, k)
 *   TM:  D = D_x at (i+1/2, k)    B = B_y at (i+1/2, j+1/2)  C = D_z at (i, j+1/2)
 * Arrays are column-major in z: field[i * nz + k].  The TE/TM split keeps
 * (D, B) of every column the 1D pair of eq. (10): for TE with b = -B_x,
 * (D_y, b) obey (10a)-(10d) exactly as (D_x, B_y) do in 1D.
 *
 * Material: the rest profile is stratified, a function of z alone.
 * eps_rest[i] holds on [i-1/2, i+1/2) and mu_rest[i] on [i, i+1) (half-open
 * cells).  A node at z reads the cell containing z - m, m = rint(beta S tau)
 * at its own time tau S (E-lattice fields at tau = n+1/2, H-lattice fields
 * at tau = n, the C field at the time of its lattice).  So the TE field B_z
 * at (i+1/2, k) reads mu_rest[k - m], and the TM field D_z at (i, j+1/2)
 * reads eps_rest[j + 1 - m] (clamped to the grid, wrapped on a z-ring).
 *
 * Per step n (state D^{n-1/2}, B^{n-1}, C^{n-1/2 or n-1}, E*^{n-1/2}):
 *   TE: B_x^n   = B_x + S (E*_y[k+1] - E*_y[k]) - bS dB_x        (10a)
 *       B_z^n   = B_z - S (E*_y[i+1] - E*_y[i]) - bS dB_z
 *       H*_x    = B_x^n / mu + beta Dbar                          (10d)
 *       H*_z    = B_z^n / mu_c
 *       D_y'    = D_y + S (H*_x[j] - H*_x[j-1]) - S (H*_z[i] - H*_z[i-1])
 *                 - bS dD_y                                        (10b)
 *       source, z ends, then E*_y = D_y'/eps + beta Bbar_x        (10c)
 *   TM: B_y^n   = B_y - S (E*_x[k+1] - E*_x[k]) + S (E*_z[i+1] - E*_z[i])
 *                 - bS dB_y                                        (10a)
 *       H*_y    = B_y^n / mu - beta Dbar_x                         (10d)
 *       D_x'    = D_x - S (H*_y[j] - H*_y[j-1]) - bS dD_x          (10b)
 *       D_z'    = D_z + S (H*_y[i] - H*_y[i-1]) - bS dD_z
 *       source, z ends, then E*_x = D_x'/eps - beta Bbar_y,
 *       E*_z = D_z'/eps_c                                          (10c)
 * with dF, Dbar, Bbar the Table 1 differences and averages along z on each
 * field's own lattice (values off the grid are the edge values) and
 * bS = beta S.  The source is the soft source of the 1D scheme on D (D_y or
 * D_x) at row src_row, src_profile[i] * g(nS) with the App. B.1 pulse g.
 * The z ends are first-order Mur on D as in 1D, per column, with the
 * normal-incidence coefficient.  Probes record the physical E (E_y =
 * E*_y - beta Bbar_x, E_x = E*_x + beta Bbar_y) at (probe_x, probe_z) at
 * t = (n+1/2) S, with the DFT of the 1D scheme.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O2_TE 0
#define O2_TM 1
#define O2_MUR1 0
#define O2_PEC 1
#define O2_PERIODIC 2

typedef struct {
    int32_t pol;
    int32_t abc;                 /* z ends                                  */
    int64_t nx, nz;
    double S, beta;
    const double *eps_rest;      /* nz                                      */
    const double *mu_rest;       /* nz                                      */
    int64_t src_row;
    const double *src_profile;   /* nx                                      */
    double src_amp, src_omega, src_t0, src_tau, src_phase, src_t_off;
    int32_t nprobe;
    const int64_t *probe_x, *probe_z;
    int32_t nfreq;
    const double *omegas;
    const double *init_d, *init_b, *init_c;   /* nx*nz each, or NULL       */
} oracle2d_problem;

typedef struct {
    double *trace;               /* nprobe*steps                            */
    double *dft_re, *dft_im;     /* nprobe*nfreq                            */
    double *final_d, *final_b, *final_c;      /* nx*nz each                 */
} oracle2d_result;

static int64_t clampi(int64_t i, int64_t lo, int64_t hi)
{
    return i < lo ? lo : (i > hi ? hi : i);
}

static int64_t wrapi(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

/* Field f of column i at lattice index k along z: wrapped on a z-ring,
 * otherwise the nearest edge value of the n nodes off the grid. */
static double atz(const double *f, int64_t i, int64_t k, int64_t nz, int64_t n, int ring)
{
    return f[i * nz + (ring ? wrapi(k, n) : clampi(k, 0, n - 1))];
}

/* Rest cell of index x - m (clamped to 0..hi, wrapped on a z-ring). */
static int64_t rest_cell(int64_t x, int64_t m, int64_t hi, int64_t nz, int ring)
{
    return ring ? wrapi(x - m, nz) : clampi(x - m, 0, hi);
}

static int64_t profile_shift(double bS, double tau)
{
    return (int64_t)rint(bS * tau);
}

/* Table 1 upwind difference along z of field f on a lattice of n nodes at
 * time level of the stored values: (dBa)/(dDa) f[k] - f[k-1] for v >= 0,
 * (dBb)/(dDb) f[k+1] - f[k] for v < 0. */
static double dz_up(const double *f, int64_t i, int64_t k, int64_t nz, int64_t n,
                    int ring, int col_a)
{
    return col_a ? f[i * nz + k] - atz(f, i, k - 1, nz, n, ring)
                 : atz(f, i, k + 1, nz, n, ring) - f[i * nz + k];
}

/* Table 1 B average at an E-lattice node k: (Ba) (B[k-1] + B[k-2])/2 for
 * v >= 0, (Bb) (B[k+1] + B[k])/2 for v < 0, on the H lattice of n nodes. */
static double b_avg(const double *B, int64_t i, int64_t k, int64_t nz, int64_t nh,
                    int ring, int col_a)
{
    if (col_a)
        return 0.5 * (atz(B, i, k - 1, nz, nh, ring) + atz(B, i, k - 2, nz, nh, ring));
    return 0.5 * (atz(B, i, k + 1, nz, nh, ring) + atz(B, i, k, nz, nh, ring));
}

/* Table 1 D average at an H-lattice node j: (Da) = (Db) (D[j+1] + D[j])/2. */
static double d_avg(const double *D, int64_t i, int64_t j, int64_t nz, int ring)
{
    return 0.5 * (atz(D, i, j + 1, nz, nz, ring) + D[i * nz + j]);
}

static double mur_coefficient(double S, double u)
{
    return (S * u - 1.0) / (S * u + 1.0);
}

int oracle2d_solve(const oracle2d_problem *p, int64_t steps, oracle2d_result *r)
{
    const int64_t nx = p->nx, nz = p->nz;
    if (nx < 1 || nz < 4 || steps < 0 || !(p->S > 0.0) || (p->pol != O2_TE && p->pol != O2_TM))
        return 1;
    const int te = (p->pol == O2_TE);
    const int ring = (p->abc == O2_PERIODIC);
    const int64_t nh = ring ? nz : nz - 1;          /* H-lattice nodes      */
    const int64_t nc = te ? nz : nh;                /* C-field nodes in z   */
    const double S = p->S, beta = p->beta, bS = beta * S;
    const int col_a = (beta >= 0.0);
    const int64_t n2 = nx * nz;

    double *D = calloc((size_t)n2, 8), *Dn = calloc((size_t)n2, 8);
    double *B = calloc((size_t)n2, 8), *Bn = calloc((size_t)n2, 8);
    double *Cf = calloc((size_t)n2, 8), *Cn = calloc((size_t)n2, 8);
    double *Es = calloc((size_t)n2, 8), *Ec = calloc((size_t)n2, 8);
    double *Hs = calloc((size_t)n2, 8), *Hc = calloc((size_t)n2, 8);
    int32_t nf = p->nfreq > 0 ? p->nfreq : 1;
    double *cw = calloc((size_t)nf, 8), *sw = calloc((size_t)nf, 8);
    if (!D || !Dn || !B || !Bn || !Cf || !Cn || !Es || !Ec || !Hs || !Hc || !cw || !sw) {
        free(D); free(Dn); free(B); free(Bn); free(Cf); free(Cn);
        free(Es); free(Ec); free(Hs); free(Hc); free(cw); free(sw);
        return 2;
    }
    if (p->init_d) memcpy(D, p->init_d, (size_t)n2 * 8);
    if (p->init_b)
        for (int64_t i = 0; i < nx; ++i)
            memcpy(B + i * nz, p->init_b + i * nz, (size_t)nh * 8);
    if (p->init_c)
        for (int64_t i = 0; i < nx; ++i)
            memcpy(Cf + i * nz, p->init_c + i * nz, (size_t)nc * 8);
    if (r->dft_re) memset(r->dft_re, 0, (size_t)p->nprobe * p->nfreq * 8);
    if (r->dft_im) memset(r->dft_im, 0, (size_t)p->nprobe * p->nfreq * 8);

    /* E*^{1/2} (and TM's E*_z) from the initial state, as (10c) leaves it. */
    {
        const int64_t mE = profile_shift(bS, 0.5);
        for (int64_t i = 0; i < nx; ++i)
            for (int64_t k = 0; k < nz; ++k) {
                const double eps = p->eps_rest[rest_cell(k, mE, nz - 1, nz, ring)];
                const double bb = b_avg(B, i, k, nz, nh, ring, col_a);
                Es[i * nz + k] = te ? D[i * nz + k] / eps + beta * bb
                                    : D[i * nz + k] / eps - beta * bb;
                if (!te && k < nc)
                    Ec[i * nz + k] = Cf[i * nz + k] /
                        p->eps_rest[rest_cell(k + 1, mE, nz - 1, nz, ring)];
            }
    }

    for (int64_t n = 1; n <= steps; ++n) {
        const int64_t mH = profile_shift(bS, (double)n);
        const int64_t mE = profile_shift(bS, (double)n + 0.5);
        /* (10a): B on the H lattice; TE also B_z on the E lattice */
        for (int64_t i = 0; i < nx; ++i) {
            const int64_t ip = (i + 1) % nx;
            for (int64_t j = 0; j < nh; ++j) {
                const double curl_z = atz(Es, i, j + 1, nz, nz, ring) - Es[i * nz + j];
                const double dB = dz_up(B, i, j, nz, nh, ring, col_a);
                if (te)
                    Bn[i * nz + j] = B[i * nz + j] + S * curl_z - bS * dB;
                else
                    Bn[i * nz + j] = B[i * nz + j] - S * curl_z
                                     + S * (Ec[ip * nz + j] - Ec[i * nz + j]) - bS * dB;
            }
            if (te)
                for (int64_t k = 0; k < nz; ++k) {
                    const double dC = dz_up(Cf, i, k, nz, nz, ring, col_a);
                    Cn[i * nz + k] = Cf[i * nz + k] - S * (Es[ip * nz + k] - Es[i * nz + k])
                                     - bS * dC;
                }
        }
        { double *t = B; B = Bn; Bn = t; }
        if (te) { double *t = Cf; Cf = Cn; Cn = t; }

        /* (10d): H* at time n */
        for (int64_t i = 0; i < nx; ++i) {
            for (int64_t j = 0; j < nh; ++j) {
                const double mu = p->mu_rest[rest_cell(j, mH, nz - 2 + ring, nz, ring)];
                const double db = d_avg(D, i, j, nz, ring);
                Hs[i * nz + j] = te ? B[i * nz + j] / mu + beta * db
                                    : B[i * nz + j] / mu - beta * db;
            }
            if (te)
                for (int64_t k = 0; k < nz; ++k)
                    Hc[i * nz + k] = Cf[i * nz + k] /
                        p->mu_rest[rest_cell(k, mH, nz - 1, nz, ring)];
        }

        /* (10b): D on the E lattice (ends replaced below); TM also D_z */
        const int64_t k0 = ring ? 0 : 1, k1 = ring ? nz : nz - 1;
        for (int64_t i = 0; i < nx; ++i) {
            const int64_t im = (i + nx - 1) % nx;
            for (int64_t k = k0; k < k1; ++k) {
                const double curl_z = Hs[i * nz + k] - atz(Hs, i, k - 1, nz, nh, ring);
                const double dD = dz_up(D, i, k, nz, nz, ring, col_a);
                if (te)
                    Dn[i * nz + k] = D[i * nz + k] + S * curl_z
                                     - S * (Hc[i * nz + k] - Hc[im * nz + k]) - bS * dD;
                else
                    Dn[i * nz + k] = D[i * nz + k] - S * curl_z - bS * dD;
            }
            if (!te)
                for (int64_t j = 0; j < nc; ++j) {
                    const double dC = dz_up(Cf, i, j, nz, nc, ring, col_a);
                    Cn[i * nz + j] = Cf[i * nz + j] + S * (Hs[i * nz + j] - Hs[im * nz + j])
                                     - bS * dC;
                }
        }

        /* soft source on D at row src_row, the App. B.1 pulse at t = nS */
        const double ts = (double)n * S;
        if (p->src_amp != 0.0 && ts <= p->src_t_off) {
            const double u = (ts - p->src_t0) / p->src_tau;
            const double g = p->src_amp * sin(p->src_omega * (ts - p->src_t0) + p->src_phase)
                             * exp(-u * u);
            for (int64_t i = 0; i < nx; ++i)
                Dn[i * nz + p->src_row] += p->src_profile[i] * g;
        }

        /* z ends at time n+1/2: first-order Mur on D per column */
        if (p->abc == O2_MUR1) {
            const double nL = sqrt(p->eps_rest[clampi(0 - mE, 0, nz - 1)] *
                                   p->mu_rest[clampi(0 - mE, 0, nz - 2)]);
            const double nR = sqrt(p->eps_rest[clampi(nz - 1 - mE, 0, nz - 1)] *
                                   p->mu_rest[clampi(nz - 2 - mE, 0, nz - 2)]);
            const double cL = mur_coefficient(S, 1.0 / nL);
            const double cR = mur_coefficient(S, 1.0 / nR);
            for (int64_t i = 0; i < nx; ++i) {
                double *dn = Dn + i * nz;
                const double *d = D + i * nz;
                dn[0] = d[1] + cL * (dn[1] - d[0]);
                dn[nz - 1] = d[nz - 2] + cR * (dn[nz - 2] - d[nz - 1]);
            }
        } else if (p->abc == O2_PEC) {
            for (int64_t i = 0; i < nx; ++i) {
                Dn[i * nz] = 0.0;
                Dn[i * nz + nz - 1] = 0.0;
            }
        }
        { double *t = D; D = Dn; Dn = t; }
        if (!te) { double *t = Cf; Cf = Cn; Cn = t; }

        /* (10c): E* at time n+1/2 */
        for (int64_t i = 0; i < nx; ++i)
            for (int64_t k = 0; k < nz; ++k) {
                const double eps = p->eps_rest[rest_cell(k, mE, nz - 1, nz, ring)];
                const double bb = b_avg(B, i, k, nz, nh, ring, col_a);
                Es[i * nz + k] = te ? D[i * nz + k] / eps + beta * bb
                                    : D[i * nz + k] / eps - beta * bb;
                if (!te && k < nc)
                    Ec[i * nz + k] = Cf[i * nz + k] /
                        p->eps_rest[rest_cell(k + 1, mE, nz - 1, nz, ring)];
            }

        /* probes: physical E at t = (n+1/2) S, trace and running DFT */
        if (p->nprobe > 0) {
            const double tp = ((double)n + 0.5) * S;
            for (int32_t m = 0; m < p->nfreq; ++m) {
                cw[m] = cos(p->omegas[m] * tp);
                sw[m] = sin(p->omegas[m] * tp);
            }
            for (int32_t q = 0; q < p->nprobe; ++q) {
                const int64_t i = p->probe_x[q], k = p->probe_z[q];
                const double bb = b_avg(B, i, k, nz, nh, ring, col_a);
                const double E = te ? Es[i * nz + k] - beta * bb : Es[i * nz + k] + beta * bb;
                if (r->trace)
                    r->trace[(int64_t)q * steps + (n - 1)] = E;
                if (r->dft_re && r->dft_im)
                    for (int32_t m = 0; m < p->nfreq; ++m) {
                        r->dft_re[q * p->nfreq + m] += E * S * cw[m];
                        r->dft_im[q * p->nfreq + m] += E * S * sw[m];
                    }
            }
        }
    }

    if (r->final_d) memcpy(r->final_d, D, (size_t)n2 * 8);
    if (r->final_b) {
        memset(r->final_b, 0, (size_t)n2 * 8);
        for (int64_t i = 0; i < nx; ++i)
            memcpy(r->final_b + i * nz, B + i * nz, (size_t)nh * 8);
    }
    if (r->final_c) {
        memset(r->final_c, 0, (size_t)n2 * 8);
        for (int64_t i = 0; i < nx; ++i)
            memcpy(r->final_c + i * nz, Cf + i * nz, (size_t)nc * 8);
    }
    free(D); free(Dn); free(B); free(Bn); free(Cf); free(Cn);
    free(Es); free(Ec); free(Hs); free(Hc); free(cw); free(sw);
    return 0;
}
