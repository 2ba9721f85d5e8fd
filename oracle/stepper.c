/*
 * FP64 reference stepper for the generalized FDTD scheme of Deck-Leger,
 * Bahrami, Li and Caloz, "Generalized FDTD Scheme for the Simulation of
 * Electromagnetic Scattering in Moving Structures" (arXiv 2304.06586).
 *
 * TEST INFRASTRUCTURE.  This file is the oracle: a plain, slow, loop-by-loop
 * statement of what the hot path computes, used only by the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark.  It shares no code,
 * header or table with the HIP library, and the library never calls it.
 *
 * Units: c = eps0 = mu0 = 1, cell size 1, time step S (Courant number,
 * Section 4 below eq. (10)), beta = v/c.
 *
 * Grid (generalized Yee cell, Section 3, Fig. 2, in 1D):
 *   E nodes k = 0..nz-1 carry D_x and the auxiliary E*_x = E_x + (v x B)_x,
 *   at half-integer times n+1/2;
 *   H nodes j = 0..nz-2 (position j+1/2) carry B_y and H*_y = H_y - (v x D)_y,
 *   at integer times n.  On a ring (periodic ends) there are nz H nodes.
 * Values outside the grid are the edge values (zero-gradient extension):
 * only the Table 1 stencils of B reach past an end, and with this reading
 * the upwind dynamic terms vanish at the first H node, so that together
 * with first-order Mur on D the ends absorb outgoing waves for either
 * sign of v.
 *
 * One time step n (state D^{n-1/2}, B^{n-1}, E*^{n-1/2} on entry), in the
 * paper's order:
 *   (10a) Faraday:  B^n  = B^{n-1} - S (E*_{j+1} - E*_j) - beta S dB
 *   (10d) H*:       H*^n = B^n / mu - beta Dbar                (modulation)
 *   (10b) Ampere:   D^{n+1/2} = D^{n-1/2} - S (H*_k - H*_{k-1}) - beta S dD
 *   source, absorbing ends
 *   (10c) E*:       E*^{n+1/2} = D^{n+1/2} / eps - beta Bbar   (modulation)
 *   probes
 * with the dynamic terms dB, dD, Bbar, Dbar of Table 1 (column a for
 * v >= 0, column b for v < 0).  For moving matter the two constitutive
 * steps use the 1D form of eq. (7) with the rest-frame tensors of the
 * footnote to eq. (5), solved for E*, H*:
 *   E* = (1-beta^2)(mu' D - beta Bbar)/(eps' mu' - beta^2)
 *   H* = (1-beta^2)(eps' B - beta Dbar)/(eps' mu' - beta^2).
 *
 * The material seen by a node is the rest profile moved by v t (eq. (5):
 * eps(r - v t)), rounded to whole cells: at time t = tau S the profile has
 * moved by m = rint(beta S tau) cells and node x reads rest cell x - m
 * (clamped to the grid, wrapped on a ring).
 *
 * Finite-duration modulation (the space-time slabs with temporal corners
 * that the footnote to the transfer-matrix method of App. B.3 sets apart):
 * when `windowed` is set, the moving profile exists only for node times t
 * with t_on <= t < t_off; at other times every node sees the uniform
 * background (eps_bg, mu_bg).  D and B carry over unchanged across the
 * switch (the temporal-interface conditions the FDTD update enforces by
 * itself, as noted in the footnote to Section 2).  Moving modulation only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MODULATION 0
#define OR_MATTER 1
#define OR_MUR1 0
#define OR_PEC 1
#define OR_PERIODIC 2

typedef struct {
    int64_t nz;
    double S;
    double beta;
    int32_t kind;
    int32_t abc;
    const double *eps_rest;    /* nz, rest permittivity of E-node cells   */
    const double *mu_rest;     /* nz, rest permeability of H-node cells   */
    int64_t src_cell;
    double src_amp, src_omega, src_t0, src_tau, src_phase, src_t_off;
    int32_t nprobe;
    const int64_t *probe_cells;
    int32_t nfreq;
    const double *omegas;
    const double *init_d;      /* optional D^{1/2}, nz                    */
    const double *init_b;      /* optional B^{0}, nz (last slot unused
                                  unless the ends are periodic)           */
    int32_t windowed;          /* 1: modulation only for t_on <= t < t_off */
    double t_on, t_off;
    double eps_bg, mu_bg;      /* the medium outside that time window     */
} oracle_problem;

typedef struct {
    double *trace;             /* nprobe*steps: E at t=(n+1/2)S, n=1..N   */
    double *dft_re;            /* nprobe*nfreq                            */
    double *dft_im;
    double *final_d;           /* nz                                      */
    double *final_b;           /* nz                                      */
    double *final_es;          /* nz                                      */
    double *final_hs;          /* nz                                      */
} oracle_result;

static int64_t clampi(int64_t i, int64_t lo, int64_t hi)
{
    return i < lo ? lo : (i > hi ? hi : i);
}

static int64_t wrapi(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

/* Value of array a (n entries) at index i: wrapped on a ring, otherwise
 * the nearest edge value off the grid. */
static double at(const double *a, int64_t i, int64_t n, int ring)
{
    if (ring)
        return a[wrapi(i, n)];
    return a[clampi(i, 0, n - 1)];
}

/* Whether the moving profile exists at node time tau*S. */
static int modulated(const oracle_problem *p, double tau)
{
    if (!p->windowed)
        return 1;
    const double t = tau * p->S;
    return t >= p->t_on && t < p->t_off;
}

/* Rest permittivity / permeability of rest cell i at node time tau*S. */
static double eps_of(const oracle_problem *p, int64_t i, double tau)
{
    return modulated(p, tau) ? p->eps_rest[i] : p->eps_bg;
}

static double mu_of(const oracle_problem *p, int64_t i, double tau)
{
    return modulated(p, tau) ? p->mu_rest[i] : p->mu_bg;
}

/* Whole-cell displacement of the moving profile at time tau*S. */
static int64_t profile_shift(double bS, double tau)
{
    return (int64_t)rint(bS * tau);
}

/* Rest cell read by lattice node x when the profile has moved by m cells;
 * hi is the last cell of that lattice. */
static int64_t rest_cell(int64_t x, int64_t m, int64_t hi, int64_t n, int ring)
{
    return ring ? wrapi(x - m, n) : clampi(x - m, 0, hi);
}

/* Table 1, the B average used in (10c): eq. (Ba) for v >= 0, (Bb) v < 0. */
static double b_average(const double *B, int64_t k, int64_t nh, int ring,
                        int col_a)
{
    if (col_a)
        return 0.5 * (at(B, k - 1, nh, ring) + at(B, k - 2, nh, ring));
    return 0.5 * (at(B, k + 1, nh, ring) + at(B, k, nh, ring));
}

/* First-order Mur coefficient for an end node whose medium has index n,
 * for a wave leaving the grid with lab speed u: (S u - 1)/(S u + 1). */
static double mur_coefficient(double S, double u)
{
    return (S * u - 1.0) / (S * u + 1.0);
}

/* Lab speed of a wave leaving through an end: 1/n for a moving
 * modulation; relativistic addition of the medium velocity for moving
 * matter (dir = +1 leaving to the right, -1 to the left). */
static double exit_speed(int kind, double n, double beta, int dir)
{
    if (kind != OR_MATTER)
        return 1.0 / n;
    double b = dir * beta;
    return (1.0 / n + b) / (1.0 + b / n);
}

int oracle_solve(const oracle_problem *p, int64_t steps, oracle_result *r)
{
    const int64_t nz = p->nz;
    if (nz < 4 || steps < 0 || !(p->S > 0.0))
        return 1;
    if (p->windowed && (p->kind != OR_MODULATION || !(p->eps_bg > 0.0) ||
                        !(p->mu_bg > 0.0)))
        return 1;
    const int ring = (p->abc == OR_PERIODIC);
    const int64_t nh = ring ? nz : nz - 1;          /* H nodes            */
    const double S = p->S;
    const double beta = p->beta;
    const double bS = beta * S;                      /* v dt / dz          */
    const int col_a = (beta >= 0.0);                 /* Table 1 column     */
    const int matter = (p->kind == OR_MATTER);
    const double b2 = beta * beta;

    double *D = calloc((size_t)nz, sizeof(double));
    double *Dn = calloc((size_t)nz, sizeof(double));
    double *B = calloc((size_t)nz, sizeof(double));
    double *Bn = calloc((size_t)nz, sizeof(double));
    double *Es = calloc((size_t)nz, sizeof(double));
    double *Hs = calloc((size_t)nz, sizeof(double));
    double *cw = calloc((size_t)(p->nfreq > 0 ? p->nfreq : 1), sizeof(double));
    double *sw = calloc((size_t)(p->nfreq > 0 ? p->nfreq : 1), sizeof(double));
    if (!D || !Dn || !B || !Bn || !Es || !Hs || !cw || !sw) {
        free(D); free(Dn); free(B); free(Bn); free(Es); free(Hs);
        free(cw); free(sw);
        return 2;
    }
    if (p->init_d)
        memcpy(D, p->init_d, (size_t)nz * sizeof(double));
    if (p->init_b)
        memcpy(B, p->init_b, (size_t)nh * sizeof(double));
    if (r->dft_re)
        memset(r->dft_re, 0, (size_t)p->nprobe * p->nfreq * sizeof(double));
    if (r->dft_im)
        memset(r->dft_im, 0, (size_t)p->nprobe * p->nfreq * sizeof(double));

    /* E*^{1/2} from the initial state, as (10c) would have left it. */
    {
        const int64_t mE = profile_shift(bS, 0.5);
        for (int64_t k = 0; k < nz; ++k) {
            const int64_t i = rest_cell(k, mE, nz - 1, nz, ring);
            const double Bbar = b_average(B, k, nh, ring, col_a);
            if (matter) {
                const double e = p->eps_rest[i], m = p->mu_rest[i];
                const double g = (1.0 - b2) / (e * m - b2);
                Es[k] = g * (m * D[k] - beta * Bbar);
            } else {
                Es[k] = D[k] / eps_of(p, i, 0.5) - beta * Bbar;
            }
        }
    }

    for (int64_t n = 1; n <= steps; ++n) {
        /* (10a) Faraday with Table 1 dB/dz at time n-1: eq. (dBa)/(dBb). */
        for (int64_t j = 0; j < nh; ++j) {
            const double dB = col_a ? B[j] - at(B, j - 1, nh, ring)
                                    : at(B, j + 1, nh, ring) - B[j];
            Bn[j] = B[j] - S * (at(Es, j + 1, nz, ring) - Es[j]) - bS * dB;
        }
        { double *t = B; B = Bn; Bn = t; }

        /* (10d) H* at time n, Table 1 D average (Da)/(Db) at n-1/2. */
        const int64_t mH = profile_shift(bS, (double)n);
        for (int64_t j = 0; j < nh; ++j) {
            const int64_t i = rest_cell(j, mH, nz - 2 + ring, nz, ring);
            const double Dbar = 0.5 * (at(D, j + 1, nz, ring) + D[j]);
            if (matter) {
                const double e = p->eps_rest[i], m = p->mu_rest[i];
                const double g = (1.0 - b2) / (e * m - b2);
                Hs[j] = g * (e * B[j] - beta * Dbar);
            } else {
                Hs[j] = B[j] / mu_of(p, i, (double)n) - beta * Dbar;
            }
        }

        /* (10b) Ampere with Table 1 dD/dz at n-1/2: eq. (dDa)/(dDb). */
        const int64_t k0 = ring ? 0 : 1, k1 = ring ? nz : nz - 1;
        for (int64_t k = k0; k < k1; ++k) {
            const double dD = col_a ? D[k] - at(D, k - 1, nz, ring)
                                    : at(D, k + 1, nz, ring) - D[k];
            Dn[k] = D[k] - S * (Hs[k] - at(Hs, k - 1, nh, ring)) - bS * dD;
        }

        /* Soft source: the modulated Gaussian of App. B.1 sampled at t=nS. */
        const double ts = (double)n * S;
        if (p->src_amp != 0.0 && ts <= p->src_t_off) {
            const double u = (ts - p->src_t0) / p->src_tau;
            Dn[p->src_cell] += p->src_amp *
                sin(p->src_omega * (ts - p->src_t0) + p->src_phase) * exp(-u * u);
        }

        /* Ends, at time n+1/2. */
        const int64_t mE = profile_shift(bS, (double)n + 0.5);
        if (p->abc == OR_MUR1) {
            const int64_t eL = clampi(0 - mE, 0, nz - 1);
            const int64_t hL = clampi(0 - mE, 0, nz - 2);
            const int64_t eR = clampi(nz - 1 - mE, 0, nz - 1);
            const int64_t hR = clampi(nz - 2 - mE, 0, nz - 2);
            const double te = (double)n + 0.5;
            const double nL = sqrt(eps_of(p, eL, te) * mu_of(p, hL, te));
            const double nR = sqrt(eps_of(p, eR, te) * mu_of(p, hR, te));
            const double cL = mur_coefficient(S, exit_speed(p->kind, nL, beta, -1));
            const double cR = mur_coefficient(S, exit_speed(p->kind, nR, beta, +1));
            Dn[0] = D[1] + cL * (Dn[1] - D[0]);
            Dn[nz - 1] = D[nz - 2] + cR * (Dn[nz - 2] - D[nz - 1]);
        } else if (p->abc == OR_PEC) {
            Dn[0] = 0.0;
            Dn[nz - 1] = 0.0;
        }
        { double *t = D; D = Dn; Dn = t; }

        /* (10c) E* at time n+1/2, Table 1 B average (Ba)/(Bb) at n. */
        for (int64_t k = 0; k < nz; ++k) {
            const int64_t i = rest_cell(k, mE, nz - 1, nz, ring);
            const double Bbar = b_average(B, k, nh, ring, col_a);
            if (matter) {
                const double e = p->eps_rest[i], m = p->mu_rest[i];
                const double g = (1.0 - b2) / (e * m - b2);
                Es[k] = g * (m * D[k] - beta * Bbar);
            } else {
                Es[k] = D[k] / eps_of(p, i, (double)n + 0.5) - beta * Bbar;
            }
        }

        /* Probes: physical E = E* + v B (inverse of eq. (2)), its trace and
         * a running DFT with kernel exp(+i w t), weight dt = S. */
        if (p->nprobe > 0) {
            const double tp = ((double)n + 0.5) * S;
            for (int32_t m = 0; m < p->nfreq; ++m) {
                cw[m] = cos(p->omegas[m] * tp);
                sw[m] = sin(p->omegas[m] * tp);
            }
            for (int32_t q = 0; q < p->nprobe; ++q) {
                const int64_t k = p->probe_cells[q];
                const double E = Es[k] + beta * b_average(B, k, nh, ring, col_a);
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

    if (r->final_d) memcpy(r->final_d, D, (size_t)nz * sizeof(double));
    if (r->final_b) {
        memset(r->final_b, 0, (size_t)nz * sizeof(double));
        memcpy(r->final_b, B, (size_t)nh * sizeof(double));
    }
    if (r->final_es) memcpy(r->final_es, Es, (size_t)nz * sizeof(double));
    if (r->final_hs) {
        memset(r->final_hs, 0, (size_t)nz * sizeof(double));
        memcpy(r->final_hs, Hs, (size_t)nh * sizeof(double));
    }
    free(D); free(Dn); free(B); free(Bn); free(Es); free(Hs);
    free(cw); free(sw);
    return 0;
}
