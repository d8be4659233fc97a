/*
 * prs_oracle.c -- plain FP64 CPU oracle for the Press-Ryden-Spergel (PRS)
 * domain-wall evolution (Correia & Martins, arXiv:1710.10420, Sec. II).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU path is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never links or calls it, and it shares no code, header or
 * constant with the HIP sources.
 *
 * Everything is double precision, written as plain loops in the order the
 * paper states the method, compiled with -ffp-contract=off so that no fused
 * multiply-add changes the rounding.  Lattice sites are stored x-fastest:
 * i = x + nx*(y + ny*z); boundaries are periodic.
 *
 * What each function follows:
 *   orc_step      Eq. (3) Laplacian, Eq. (4) velocity kick, Eq. (5) drift,
 *                 Eq. (6) damping coefficient; the force of Eq. (2) carries the
 *                 scale-factor power a^beta (beta = 0 for the PRS choice, where
 *                 Eq. (4) is printed without it).
 *   orc_stats     Eq. (7) wall area per unit volume from sign-changing links
 *                 and Eq. (8) (gamma v)^2 over the sites that hold walls.
 *   orc_energy    discrete flat-space energy used as an invariant check.
 *   orc_adjoint   reverse-mode derivative of repeated orc_step applications
 *                 (hand derived from Eqs. (3)-(6)), with its own plain
 *                 store-every-K / recompute checkpointing.
 *
 * Readings taken where the paper is silent (each is listed with its reason
 * in the design notes of the repository):
 *   - Eq. (3) carries no 1/dx^2; it is included here (dx = 1 leaves it exact).
 *   - delta of Eq. (6) is evaluated at eta_n = eta0 + n*deta, the time at
 *     which the force of step n is evaluated; d ln a / d ln eta = m constant.
 *   - a link crosses a wall when (phi_i >= 0) != (phi_j >= 0); every forward
 *     link (site, +e_d) is visited once.
 *   - the gradient in the area weight of Eq. (7) is the centred difference at
 *     the link's lower-index site; a site with zero gradient gets weight 1.
 *   - E_k in Eq. (8) is phi_dot^2, so each wall site contributes
 *     (1/2) phi_dot^2 / V; a wall site is a site touching at least one
 *     crossing link; sites with V = 0 add nothing but are still counted.
 *   - diagnostics of state n use (phi^n, phi_dot^{n-1/2}).
 *   - the scale factor is a(eta) = (eta/eta0)^m, so a = 1 at the start; with
 *     beta != 0 the force of step n is a(eta_n)^beta dV/dphi, and the
 *     potential energy of a wall in Eq. (8) is a(eta_n)^beta V (a static
 *     wall then has (1/2) phi'^2 = a^beta V, and a boosted one still gives
 *     (gamma v)^2).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t ndim;      /* 2 or 3 */
    int32_t reserved;
    int64_t n[3];      /* lattice sides (x, y, z); n[2] is ignored in 2D */
    double dx;         /* lattice spacing */
    double deta;       /* conformal time step */
    double eta0;       /* conformal time of step 0 */
    double alpha;      /* damping coefficient of Eq. (2) */
    double m;          /* d ln a / d ln eta (constant era exponent) */
    double V0;         /* potential height of Eq. (1) */
    double W0;         /* wall thickness parameter, V0 = pi^2/(2 W0^2) */
    double phi0;       /* vacuum value of Eq. (1) */
    double beta;       /* scale-factor power of the force in Eq. (2) */
} orc_params;

typedef struct {
    int64_t step;
    double eta;
    uint64_t links;          /* crossing forward links, all directions */
    uint64_t links_dir[3];   /* crossing forward links per direction */
    uint64_t wall_sites;     /* sites touching a crossing link */
    uint64_t nonfinite;      /* sites where phi or phi_dot is not finite */
    double area_density;     /* rho = A / V of Eq. (7) */
    double gv2;              /* (gamma v)^2 of Eq. (8) */
} orc_record;

static int64_t sites_of(const orc_params *p)
{
    return p->n[0] * p->n[1] * (p->ndim == 3 ? p->n[2] : 1);
}

static int64_t wrap(int64_t v, int64_t n)
{
    v %= n;
    return v < 0 ? v + n : v;
}

/* Index of the neighbour of site (x,y,z) displaced by s (+1/-1) along axis d. */
static int64_t neighbour(const orc_params *p, int64_t x, int64_t y, int64_t z,
                         int d, int s)
{
    int64_t nx = p->n[0], ny = p->n[1], nz = p->ndim == 3 ? p->n[2] : 1;
    if (d == 0) x = wrap(x + s, nx);
    if (d == 1) y = wrap(y + s, ny);
    if (d == 2) z = wrap(z + s, nz);
    return x + nx * (y + ny * z);
}

/* Eq. (3) and its 3D extension: sum over axes of both neighbours minus
 * 2*D times the centre, divided by dx^2. */
static double laplacian_at(const orc_params *p, const double *f,
                           int64_t x, int64_t y, int64_t z)
{
    int64_t nx = p->n[0], ny = p->n[1];
    int64_t i = x + nx * (y + ny * z);
    double acc = 0.0;
    for (int d = 0; d < p->ndim; ++d)
        acc += f[neighbour(p, x, y, z, d, +1)] + f[neighbour(p, x, y, z, d, -1)];
    acc -= 2.0 * p->ndim * f[i];
    return acc / (p->dx * p->dx);
}

/* dV/dphi for V = V0 (phi^2/phi0^2 - 1)^2  (Eq. 1). */
static double dV(const orc_params *p, double f)
{
    double q = f * f / (p->phi0 * p->phi0) - 1.0;
    return 4.0 * p->V0 * f * q / (p->phi0 * p->phi0);
}

/* d^2V/dphi^2. */
static double d2V(const orc_params *p, double f)
{
    return 4.0 * p->V0 * (3.0 * f * f / (p->phi0 * p->phi0) - 1.0) / (p->phi0 * p->phi0);
}

/* V(phi) of Eq. (1). */
static double Vpot(const orc_params *p, double f)
{
    double q = f * f / (p->phi0 * p->phi0) - 1.0;
    return p->V0 * q * q;
}

/* When set, the long-running loops print one line per segment to stdout
 * (progress of full-length runs; no effect on any result). */
static int orc_progress = 0;

void orc_set_progress(int on)
{
    orc_progress = on;
}

double orc_eta(const orc_params *p, int64_t n)
{
    return p->eta0 + (double)n * p->deta;
}

/* Eq. (6) at step n. */
double orc_delta(const orc_params *p, int64_t n)
{
    return 0.5 * p->alpha * (p->deta / orc_eta(p, n)) * p->m;
}

/* a(eta_n)^beta with a(eta) = (eta/eta0)^m: the factor of the force in
 * Eq. (2) at step n (exactly 1 for beta = 0). */
double orc_force_scale(const orc_params *p, int64_t n)
{
    if (p->beta == 0.0) return 1.0;
    return pow(pow(orc_eta(p, n) / p->eta0, p->m), p->beta);
}

/* One PRS step n -> n+1 (Eqs. 3-5).  phi holds phi^n (read only), pi holds
 * phi_dot^{n-1/2} on entry and phi_dot^{n+1/2} on exit, phi_next receives
 * phi^{n+1}.  Every site reads the old phi^n (Jacobi update). */
void orc_step(const orc_params *p, int64_t n, const double *phi, double *pi,
              double *phi_next)
{
    int64_t nx = p->n[0], ny = p->n[1], nz = p->ndim == 3 ? p->n[2] : 1;
    double delta = orc_delta(p, n);
    double deta = p->deta;
    double A = orc_force_scale(p, n);
#pragma omp parallel for schedule(static)
    for (int64_t zy = 0; zy < ny * nz; ++zy) {
        int64_t y = zy % ny, z = zy / ny;
        for (int64_t x = 0; x < nx; ++x) {
            int64_t i = x + nx * (y + ny * z);
            double lap = laplacian_at(p, phi, x, y, z);
            double kick = (1.0 - delta) * pi[i] + deta * (lap - A * dV(p, phi[i]));
            pi[i] = kick / (1.0 + delta);                 /* Eq. (4) */
            phi_next[i] = phi[i] + deta * pi[i];          /* Eq. (5) */
        }
    }
}

/* Diagnostics of Eqs. (7) and (8) on the state (phi, pi). */
void orc_stats(const orc_params *p, int64_t n, const double *phi, const double *pi,
               orc_record *out)
{
    int64_t nx = p->n[0], ny = p->n[1], nz = p->ndim == 3 ? p->n[2] : 1;
    int64_t rows = ny * nz;
    /* per-row partial results, summed in row order afterwards so the result
     * does not depend on the thread count */
    uint64_t *rl = calloc((size_t)rows * 6, sizeof(uint64_t));
    double *rf = calloc((size_t)rows * 2, sizeof(double));
    double A = orc_force_scale(p, n);
#pragma omp parallel for schedule(static)
    for (int64_t zy = 0; zy < rows; ++zy) {
        int64_t y = zy % ny, z = zy / ny;
        uint64_t ldir[3] = {0, 0, 0}, walls = 0, bad = 0;
        double area = 0.0, ek = 0.0;
        for (int64_t x = 0; x < nx; ++x) {
            int64_t i = x + nx * (y + ny * z);
            int si = phi[i] >= 0.0;
            if (!isfinite(phi[i]) || !isfinite(pi[i])) bad++;
            double gsq = 0.0, gabs = 0.0;
            int crossings = 0, wall = 0;
            for (int d = 0; d < p->ndim; ++d) {
                int64_t jf = neighbour(p, x, y, z, d, +1);
                int64_t jb = neighbour(p, x, y, z, d, -1);
                double g = (phi[jf] - phi[jb]) / (2.0 * p->dx);
                gsq += g * g;
                gabs += fabs(g);
                int sf = phi[jf] >= 0.0, sb = phi[jb] >= 0.0;
                if (si != sf) { ldir[d]++; crossings++; wall = 1; }
                if (sb != si) wall = 1;
            }
            if (crossings) {
                double w = gabs > 0.0 ? sqrt(gsq) / gabs : 1.0;
                area += (double)crossings * w;
            }
            if (wall) {
                walls++;
                double V = A * Vpot(p, phi[i]);
                if (V > 0.0) ek += 0.5 * pi[i] * pi[i] / V;
            }
        }
        for (int d = 0; d < 3; ++d) rl[zy * 6 + d] = ldir[d];
        rl[zy * 6 + 3] = walls;
        rl[zy * 6 + 4] = bad;
        rf[zy * 2 + 0] = area;
        rf[zy * 2 + 1] = ek;
    }
    memset(out, 0, sizeof(*out));
    double area = 0.0, ek = 0.0;
    for (int64_t r = 0; r < rows; ++r) {
        for (int d = 0; d < 3; ++d) out->links_dir[d] += rl[r * 6 + d];
        out->wall_sites += rl[r * 6 + 3];
        out->nonfinite += rl[r * 6 + 4];
        area += rf[r * 2 + 0];
        ek += rf[r * 2 + 1];
    }
    out->links = out->links_dir[0] + out->links_dir[1] + out->links_dir[2];
    out->step = n;
    out->eta = orc_eta(p, n);
    /* Eq. (7): Delta A = dx^(D-1) per link, V = sites * dx^D */
    double dA = pow(p->dx, p->ndim - 1);
    double vol = (double)sites_of(p) * pow(p->dx, p->ndim);
    out->area_density = dA * area / vol;
    /* Eq. (8) */
    out->gv2 = out->wall_sites ? ek / (double)out->wall_sites : 0.0;
    free(rl);
    free(rf);
}

/* Advance nsteps from global step n0.  A diagnostic record of state n is
 * written for every n in [n0, n0+nsteps) with n % diag_every == 0 (if
 * diag_every > 0), up to cap records.  Returns the number of records. */
int64_t orc_run(const orc_params *p, int64_t n0, int64_t nsteps, int32_t diag_every,
                double *phi, double *pi, orc_record *series, int64_t cap)
{
    int64_t N = sites_of(p), written = 0;
    double *tmp = malloc((size_t)N * sizeof(double));
    double *cur = phi, *next = tmp;       /* ping-pong: phi^n in cur */
    for (int64_t k = 0; k < nsteps; ++k) {
        int64_t n = n0 + k;
        if (diag_every > 0 && n % diag_every == 0 && written < cap && series)
            orc_stats(p, n, cur, pi, &series[written++]);
        orc_step(p, n, cur, pi, next);
        double *t = cur; cur = next; next = t;
    }
    if (cur != phi) memcpy(phi, cur, (size_t)N * sizeof(double));
    free(tmp);
    return written;
}

/* Discrete flat-space energy at integer step n:
 * sum_i [ 1/2 pi^{n-1/2} pi^{n+1/2} + 1/2 sum_d (phi_{i+e_d}-phi_i)^2/dx^2 + V(phi_i) ]
 * times the cell volume dx^D.  With alpha = 0 it is a conserved quantity of
 * the leapfrog for a quadratic potential. */
double orc_energy(const orc_params *p, const double *phi, const double *pi_prev,
                  const double *pi_next)
{
    int64_t nx = p->n[0], ny = p->n[1], nz = p->ndim == 3 ? p->n[2] : 1;
    double e = 0.0;
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t i = x + nx * (y + ny * z);
                double grad = 0.0;
                for (int d = 0; d < p->ndim; ++d) {
                    double df = (phi[neighbour(p, x, y, z, d, +1)] - phi[i]) / p->dx;
                    grad += df * df;
                }
                e += 0.5 * pi_prev[i] * pi_next[i] + 0.5 * grad + Vpot(p, phi[i]);
            }
    return e * pow(p->dx, p->ndim);
}

/* Loss of the differentiable path: sum over sites of V(phi)/V0
 * = (phi^2/phi0^2 - 1)^2. */
double orc_loss(const orc_params *p, const double *phi)
{
    int64_t N = sites_of(p);
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        double q = phi[i] * phi[i] / (p->phi0 * p->phi0) - 1.0;
        s += q * q;
    }
    return s;
}

/* Reverse-mode derivative of nsteps PRS steps started at global step n0 from
 * (phi0, pi0), for the loss orc_loss of the final field.
 *
 * Let w be the total adjoint of phi_dot^{n+1/2}.  Step n reads phi^n and
 * phi_dot^{n-1/2}, so with mu = dL/dphi^{n+1} and nu the adjoint of
 * phi_dot^{n+1/2} from later steps:
 *     w        = nu + deta * mu                          (from Eq. 5)
 *     dL/dphi^n = mu + b_n (Lap^T w - A_n V''(phi^n) w)  (from Eqs. 3, 4)
 *     nu'      = a_n w                                   (from Eq. 4)
 *     dL/dV0  += -b_n A_n sum_i w_i * d(V'(phi_i))/dV0
 * with a_n = (1-delta_n)/(1+delta_n), b_n = deta/(1+delta_n), A_n the
 * force's scale-factor power a(eta_n)^beta; the periodic
 * Laplacian is symmetric, so Lap^T = Lap.
 *
 * Checkpointing: (phi, pi) is stored every ckpt_every steps on the way
 * forward; each segment is recomputed from its checkpoint, keeping every
 * phi^n of the segment, and then swept backwards.
 *
 * Outputs: grad_phi = dL/dphi^{n0}, grad_pi = dL/dphi_dot^{n0-1/2},
 * *dL_dV0 and *loss.  Returns 0, or -1 on allocation failure. */
int orc_adjoint(const orc_params *p, int64_t n0, int64_t nsteps, int32_t ckpt_every,
                const double *phi0, const double *pi0, double *grad_phi,
                double *grad_pi, double *dL_dV0, double *loss)
{
    int64_t N = sites_of(p);
    int64_t K = ckpt_every > 0 ? ckpt_every : 1;
    int64_t nseg = nsteps > 0 ? (nsteps + K - 1) / K : 0;
    size_t fb = (size_t)N * sizeof(double);
    double *ck_phi = malloc(fb * (size_t)(nseg ? nseg : 1));
    double *ck_pi = malloc(fb * (size_t)(nseg ? nseg : 1));
    double *phi = malloc(fb), *pi = malloc(fb), *tmp = malloc(fb);
    double *traj = malloc(fb * (size_t)(K + 1));
    double *w = malloc(fb), *mu = malloc(fb), *nu = malloc(fb);
    int64_t nx = p->n[0], ny = p->n[1], nz = p->ndim == 3 ? p->n[2] : 1;
    double *rowg = malloc((size_t)(ny * nz) * sizeof(double));
    if (!ck_phi || !ck_pi || !phi || !pi || !tmp || !traj || !w || !mu || !nu || !rowg) {
        free(ck_phi); free(ck_pi); free(phi); free(pi); free(tmp);
        free(traj); free(w); free(mu); free(nu); free(rowg);
        return -1;
    }
    memcpy(phi, phi0, fb);
    memcpy(pi, pi0, fb);

    /* forward sweep with checkpoints (phi and tmp swap roles each step) */
    for (int64_t s = 0; s < nseg; ++s) {
        memcpy(ck_phi + (size_t)s * N, phi, fb);
        memcpy(ck_pi + (size_t)s * N, pi, fb);
        int64_t len = (s + 1) * K <= nsteps ? K : nsteps - s * K;
        for (int64_t k = 0; k < len; ++k) {
            orc_step(p, n0 + s * K + k, phi, pi, tmp);
            double *t = phi; phi = tmp; tmp = t;
        }
    }
    *loss = orc_loss(p, phi);

    /* seed: dL/dphi^S = 4 phi (phi^2/phi0^2 - 1)/phi0^2; phi_dot^{S-1/2} does
     * not enter the loss */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double q = phi[i] * phi[i] / (p->phi0 * p->phi0) - 1.0;
        mu[i] = 4.0 * phi[i] * q / (p->phi0 * p->phi0);
        nu[i] = 0.0;
    }
    double G = 0.0;
    double dVp_dV0_scale = 4.0 / (p->phi0 * p->phi0);   /* d(V')/dV0 = V'/V0 */

    for (int64_t s = nseg - 1; s >= 0; --s) {
        int64_t len = (s + 1) * K <= nsteps ? K : nsteps - s * K;
        if (orc_progress)
            fprintf(stdout, "oracle adjoint: segment %lld of %lld\n", (long long)(nseg - s), (long long)nseg),
                fflush(stdout);
        /* recompute phi^n for the segment */
        memcpy(traj, ck_phi + (size_t)s * N, fb);
        memcpy(pi, ck_pi + (size_t)s * N, fb);
        for (int64_t k = 0; k + 1 < len; ++k)
            orc_step(p, n0 + s * K + k, traj + (size_t)k * N, pi, traj + (size_t)(k + 1) * N);
        for (int64_t k = len - 1; k >= 0; --k) {
            int64_t n = n0 + s * K + k;
            const double *ph = traj + (size_t)k * N;
            double delta = orc_delta(p, n);
            double a = (1.0 - delta) / (1.0 + delta);
            double b = p->deta / (1.0 + delta);
            double A = orc_force_scale(p, n);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) w[i] = nu[i] + p->deta * mu[i];
#pragma omp parallel for schedule(static)
            for (int64_t zy = 0; zy < ny * nz; ++zy) {
                int64_t y = zy % ny, z = zy / ny;
                double g = 0.0;
                for (int64_t x = 0; x < nx; ++x) {
                    int64_t i = x + nx * (y + ny * z);
                    double lw = laplacian_at(p, w, x, y, z);
                    mu[i] = mu[i] + b * (lw - A * d2V(p, ph[i]) * w[i]);
                    double q = ph[i] * ph[i] / (p->phi0 * p->phi0) - 1.0;
                    g += w[i] * dVp_dV0_scale * ph[i] * q;
                }
                rowg[zy] = g;
            }
            double g = 0.0;
            for (int64_t r = 0; r < ny * nz; ++r) g += rowg[r];
            g *= A;
            G -= b * g;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < N; ++i) nu[i] = a * w[i];
        }
    }
    memcpy(grad_phi, mu, fb);
    memcpy(grad_pi, nu, fb);
    *dL_dV0 = G;
    free(ck_phi); free(ck_pi); free(phi); free(pi); free(tmp);
    free(traj); free(w); free(mu); free(nu); free(rowg);
    return 0;
}
