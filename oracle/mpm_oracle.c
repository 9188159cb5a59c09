/*
 * Plain FP64 CPU oracle for one explicit MLS-MPM substep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP library.
 *
 * What it computes (paper: "Material Point Method on a Single GPU", the five
 * phases rebuild-mapping / sort / P2G / grid update / G2P):
 *   - binning: particle code (block code in the high bits, cell code in the
 *     low bits, 3-D interleaved), a stable sort by that code, the particle
 *     ("geometric") blocks and their 3x3x3 dilation ("physical" blocks), and
 *     the free-zone test of the rebuild-mapping subsection;
 *   - P2G / grid update / G2P as textbook MLS-MPM with APIC and quadratic
 *     B-splines on a DENSE grid of (n+1)^3 nodes, particles in input order.
 * The paper cites MLS-MPM (Results section) but does not write its equations;
 * the forms used here are the standard ones and every reading is listed in the
 * design notes.  The sparse blocks, free zone, sorting and tiling of the GPU
 * path all reach this dense result up to floating-point summation order.
 *
 * Layout conventions (shared only as a documented data format):
 *   particle arrays are structure-of-arrays: x[3][N], v[3][N], C[9][N],
 *   F[9][N] with matrix entry (a,b) at component a*3+b, s[N] (J_P for snow,
 *   1 + q, q the hardening state, for sand,
 *   J for water, unused for jelly).  Dense grid node (i,j,k) sits at
 *   (i,j,k)*dx and is stored at ((i*(n+1))+j)*(n+1)+k; vector grid fields are
 *   [3][(n+1)^3].
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int kind; /* 0 fixed-corotated jelly, 1 snow (clamped SVD + hardening), 2 water,
                 3 sand (Hencky elasticity, Drucker-Prager return map with hardening) */
    double E, nu, rho, ppc, theta_c, theta_s, xi, bulk;
    double h0, h1, h2, h3; /* sand friction angle (degrees) phi(q) = h0 + (h1 q - h3) exp(-h2 q) */
} om_material;

typedef struct {
    int n;         /* cells per axis on the unit cube, dx = 1/n */
    int bc;        /* 0 sticky, 1 slip, 2 separating slip */
    int bc_cells;  /* wall thickness in cells */
    double gravity[3];
    double dt;
} om_config;

enum { OM_JELLY = 0, OM_SNOW = 1, OM_WATER = 2, OM_SAND = 3 };

/* ---------------------------------------------------------------- 3x3 util */
static void mat_mul(const double A[9], const double B[9], double out[9]) {
    double r[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += A[a * 3 + k] * B[k * 3 + b];
            r[a * 3 + b] = acc;
        }
    memcpy(out, r, sizeof r);
}

static void mat_mul_bt(const double A[9], const double B[9], double out[9]) { /* A * B^T */
    double r[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += A[a * 3 + k] * B[b * 3 + k];
            r[a * 3 + b] = acc;
        }
    memcpy(out, r, sizeof r);
}

static double mat_det(const double A[9]) {
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* -------------------------------------------------------------- 3x3 SVD
 * One-sided (Hestenes) Jacobi: right-multiply A = F by plane rotations until
 * its columns are mutually orthogonal; then A = U*Sigma and F = U Sigma V^T.
 * Convention: sigma sorted descending, U and V proper rotations, and the sign
 * of det F carried by the smallest singular value.                           */
void om_svd3(const double F[9], double U[9], double S[3], double V[9]) {
    double A[9];
    memcpy(A, F, sizeof A);
    double W[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    static const int P[3] = {0, 0, 1}, Q[3] = {1, 2, 2};
    for (int sweep = 0; sweep < 80; ++sweep) {
        double worst = 0.0;
        for (int r = 0; r < 3; ++r) {
            int p = P[r], q = Q[r];
            double alpha = 0, beta = 0, gamma = 0;
            for (int i = 0; i < 3; ++i) {
                alpha += A[i * 3 + p] * A[i * 3 + p];
                beta += A[i * 3 + q] * A[i * 3 + q];
                gamma += A[i * 3 + p] * A[i * 3 + q];
            }
            double scale = sqrt(alpha * beta);
            if (gamma == 0.0 || scale == 0.0) continue;
            double rel = fabs(gamma) / scale;
            if (rel > worst) worst = rel;
            if (rel < 1e-17) continue;
            double zeta = (beta - alpha) / (2.0 * gamma);
            double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
            for (int i = 0; i < 3; ++i) {
                double ap = A[i * 3 + p], aq = A[i * 3 + q];
                A[i * 3 + p] = c * ap - s * aq;
                A[i * 3 + q] = s * ap + c * aq;
                double vp = W[i * 3 + p], vq = W[i * 3 + q];
                W[i * 3 + p] = c * vp - s * vq;
                W[i * 3 + q] = s * vp + c * vq;
            }
        }
        if (worst < 1e-15) break;
    }
    double sig[3];
    for (int k = 0; k < 3; ++k)
        sig[k] = sqrt(A[0 * 3 + k] * A[0 * 3 + k] + A[1 * 3 + k] * A[1 * 3 + k] + A[2 * 3 + k] * A[2 * 3 + k]);
    int ord[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (sig[ord[j]] > sig[ord[i]]) { int tmp = ord[i]; ord[i] = ord[j]; ord[j] = tmp; }
    double Uo[9], Vo[9], So[3];
    for (int k = 0; k < 3; ++k) {
        int src = ord[k];
        So[k] = sig[src];
        for (int i = 0; i < 3; ++i) {
            Vo[i * 3 + k] = W[i * 3 + src];
            Uo[i * 3 + k] = (sig[src] > 0) ? A[i * 3 + src] / sig[src] : 0.0;
        }
    }
    /* complete U where a singular value vanished */
    double tiny = 1e-300 + 1e-14 * So[0];
    if (So[1] <= tiny) { /* rank <= 1: build any orthonormal completion of U col 0 */
        double a[3] = {Uo[0], Uo[3], Uo[6]};
        if (So[0] <= tiny) { a[0] = 1; a[1] = 0; a[2] = 0; Uo[0] = 1; Uo[3] = 0; Uo[6] = 0; }
        double e[3] = {0, 0, 0};
        int m = (fabs(a[0]) < fabs(a[1])) ? ((fabs(a[0]) < fabs(a[2])) ? 0 : 2) : ((fabs(a[1]) < fabs(a[2])) ? 1 : 2);
        e[m] = 1.0;
        double b[3] = {a[1] * e[2] - a[2] * e[1], a[2] * e[0] - a[0] * e[2], a[0] * e[1] - a[1] * e[0]};
        double nb = sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
        for (int i = 0; i < 3; ++i) Uo[i * 3 + 1] = b[i] / nb;
    }
    if (So[2] <= tiny) {
        double a[3] = {Uo[0], Uo[3], Uo[6]}, b[3] = {Uo[1], Uo[4], Uo[7]};
        Uo[2] = a[1] * b[2] - a[2] * b[1];
        Uo[5] = a[2] * b[0] - a[0] * b[2];
        Uo[8] = a[0] * b[1] - a[1] * b[0];
    }
    if (mat_det(Vo) < 0) {
        for (int i = 0; i < 3; ++i) { Vo[i * 3 + 2] = -Vo[i * 3 + 2]; Uo[i * 3 + 2] = -Uo[i * 3 + 2]; }
    }
    if (mat_det(Uo) < 0) {
        for (int i = 0; i < 3; ++i) Uo[i * 3 + 2] = -Uo[i * 3 + 2];
        So[2] = -So[2];
    }
    memcpy(U, Uo, sizeof Uo);
    memcpy(V, Vo, sizeof Vo);
    memcpy(S, So, sizeof So);
}

/* ------------------------------------------------------- constitutive laws */
static void lame(const om_material* m, double* mu, double* la) {
    *mu = m->E / (2.0 * (1.0 + m->nu));
    *la = m->E * m->nu / ((1.0 + m->nu) * (1.0 - 2.0 * m->nu));
}

/* Fixed-corotated Kirchhoff stress: tau = 2 mu (F - R) F^T + lambda (J-1) J I,
 * R the rotation of the polar decomposition (R = U V^T), J = det F.          */
void om_fixed_corotated(const double F[9], double mu, double la, double tau[9]) {
    double U[9], S[3], V[9], R[9], FmR[9];
    om_svd3(F, U, S, V);
    mat_mul_bt(U, V, R);
    for (int i = 0; i < 9; ++i) FmR[i] = F[i] - R[i];
    mat_mul_bt(FmR, F, tau);
    double J = mat_det(F);
    for (int i = 0; i < 9; ++i) tau[i] *= 2.0 * mu;
    for (int a = 0; a < 3; ++a) tau[a * 3 + a] += la * (J - 1.0) * J;
}

/* Hencky (St. Venant-Kirchhoff in logarithmic strain) Kirchhoff stress, the
 * elasticity of the Drucker-Prager sand of Klar et al. 2016 (the sand model
 * the paper uses is not given in it; this one stands in).  With
 * F = U diag(sig) V^T and eps_k = log sig_k the energy is
 * psi = mu sum eps_k^2 + la/2 (sum eps_k)^2, whose Kirchhoff stress is
 * tau = U diag(2 mu eps_k + la sum eps) U^T.  The sign an inverted gradient
 * gives its smallest singular value is dropped (eps_k = log |sig_k|, and
 * |sig_k| is floored at OM_SAND_SIG_FLOOR).                                  */
#define OM_SAND_SIG_FLOOR 1e-6
static double sand_log(double sig) {
    double a = fabs(sig);
    return log(a > OM_SAND_SIG_FLOOR ? a : OM_SAND_SIG_FLOOR);
}

void om_hencky(const double F[9], double mu, double la, double tau[9]) {
    double U[9], S[3], V[9], e[3];
    om_svd3(F, U, S, V);
    for (int k = 0; k < 3; ++k) e[k] = sand_log(S[k]);
    double tr = e[0] + e[1] + e[2];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += U[a * 3 + k] * (2.0 * mu * e[k] + la * tr) * U[b * 3 + k];
            tau[a * 3 + b] = acc;
        }
}

/* Drucker-Prager friction coefficient of hardening state q: the friction
 * angle phi = h0 + (h1 q - h3) exp(-h2 q) degrees, and
 * alpha = sqrt(2/3) * 2 sin(phi) / (3 - sin(phi)), the cone that matches the
 * Mohr-Coulomb surface of angle phi in triaxial compression.               */
double om_sand_alpha(const om_material* m, double q) {
    const double pi = 3.14159265358979323846;
    double phi = (m->h0 + (m->h1 * q - m->h3) * exp(-m->h2 * q)) * pi / 180.0;
    double sp = sin(phi);
    return sqrt(2.0 / 3.0) * 2.0 * sp / (3.0 - sp);
}

/* Sand return map (Klar et al. 2016, in logarithmic strain): with
 * eps = log sig of the trial gradient, its trace t and deviator d,
 *   t > 0 (expansion): all elastic strain is released (eps' = 0) and the
 *     hardening state grows by |eps|;
 *   else, with dg = |d| + (3 la + 2 mu)/(2 mu) t alpha(q):
 *     dg <= 0: the state is inside the cone and unchanged (Fe = Fhat, so an
 *       inverted gradient stays inverted: only the two plastic branches
 *       rebuild the gradient from its singular values);
 *     dg > 0: the deviator shrinks along itself by dg (eps' = eps - dg d/|d|,
 *       the trace, i.e. the volume, is kept) and q grows by dg.
 * Fe = U diag(exp eps') V^T; q_out the new hardening state.                */
void om_sand_project(const om_material* m, const double Fhat[9], double q, double Fe[9], double* q_out) {
    double mu, la, U[9], S[3], V[9], e[3], en[3], US[9];
    lame(m, &mu, &la);
    om_svd3(Fhat, U, S, V);
    for (int k = 0; k < 3; ++k) e[k] = sand_log(S[k]);
    double t = e[0] + e[1] + e[2];
    double d[3], nd = 0.0, ne = 0.0;
    for (int k = 0; k < 3; ++k) {
        d[k] = e[k] - t / 3.0;
        nd += d[k] * d[k];
        ne += e[k] * e[k];
    }
    nd = sqrt(nd);
    ne = sqrt(ne);
    double dq = 0.0;
    if (t > 0.0) {
        for (int k = 0; k < 3; ++k) en[k] = 0.0;
        dq = ne;
    } else {
        double dg = nd + (3.0 * la + 2.0 * mu) / (2.0 * mu) * t * om_sand_alpha(m, q);
        if (dg <= 0.0) {
            for (int i = 0; i < 9; ++i) Fe[i] = Fhat[i];
            *q_out = q;
            return;
        } else {
            for (int k = 0; k < 3; ++k) en[k] = e[k] - dg * d[k] / nd;
            dq = dg;
        }
    }
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) US[i * 3 + k] = U[i * 3 + k] * exp(en[k]);
    mat_mul_bt(US, V, Fe);
    *q_out = q + dq;
}

/* Kirchhoff stress of the stored particle state.                            */
void om_stress(const om_material* m, const double F[9], double s, double tau[9]) {
    double mu, la;
    lame(m, &mu, &la);
    if (m->kind == OM_JELLY) {
        om_fixed_corotated(F, mu, la, tau);
    } else if (m->kind == OM_SNOW) {
        double h = exp(m->xi * (1.0 - s)); /* hardening from the plastic volume J_P */
        om_fixed_corotated(F, mu * h, la * h, tau);
    } else if (m->kind == OM_SAND) {
        om_hencky(F, mu, la, tau);
    } else { /* water: psi = K/2 (J-1)^2, tau = J dpsi/dJ I */
        double J = s;
        for (int i = 0; i < 9; ++i) tau[i] = 0.0;
        for (int a = 0; a < 3; ++a) tau[a * 3 + a] = m->bulk * (J - 1.0) * J;
    }
}

/* Snow return map: clamp the singular values of the trial elastic gradient
 * into [1-theta_c, 1+theta_s]; the removed volume goes to J_P.              */
void om_snow_project(const om_material* m, const double Fhat[9], double Jp, double Fe[9], double* Jp_out) {
    double U[9], S[3], V[9], Sc[3], US[9];
    om_svd3(Fhat, U, S, V);
    double lo = 1.0 - m->theta_c, hi = 1.0 + m->theta_s;
    for (int k = 0; k < 3; ++k) Sc[k] = S[k] < lo ? lo : (S[k] > hi ? hi : S[k]);
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) US[i * 3 + k] = U[i * 3 + k] * Sc[k];
    mat_mul_bt(US, V, Fe);
    *Jp_out = Jp * (S[0] * S[1] * S[2]) / (Sc[0] * Sc[1] * Sc[2]);
}

/* ---------------------------------------------------------------- weights
 * Quadratic B-spline stencil along one axis: t = x/dx, base = floor(t - 1/2),
 * f = t - base in [1/2, 3/2); weights of nodes base, base+1, base+2.         */
void om_weights(double t, int* base, double w[3]) {
    double b = floor(t - 0.5);
    double f = t - b;
    *base = (int)b;
    w[0] = 0.5 * (1.5 - f) * (1.5 - f);
    w[1] = 0.75 - (f - 1.0) * (f - 1.0);
    w[2] = 0.5 * (f - 0.5) * (f - 0.5);
}

static long node_index(int n, int i, int j, int k) { return ((long)i * (n + 1) + j) * (n + 1) + k; }

/* ------------------------------------------------------------------- P2G
 * m_i = sum_p w_ip m_p,  p_i = sum_p w_ip (m_p v_p + A_p (x_i - x_p)),
 * A_p = m_p C_p - (4 dt V0 / dx^2) tau_p.  Particles whose stencil leaves the
 * node range [0, n] are skipped and counted.                                 */

/* Stencil of particle p (base node, weights, f = x/dx - base per axis) and
 * its affine momentum matrix A_p.  Returns 1 if the stencil leaves the grid. */
static int p2g_prepare(const om_config* cfg, const om_material* mat, long N, long p, const double* x,
                       const double* C, const double* F, const double* s, int base[3], double w[3][3],
                       double f[3], double A[9]) {
    const int n = cfg->n;
    const double dx = 1.0 / n;
    const double V0 = dx * dx * dx / mat->ppc;
    const double mp = mat->rho * V0;
    double Fp[9], Cp[9], tau[9];
    for (int c = 0; c < 9; ++c) { Fp[c] = F ? F[c * N + p] : (c % 4 == 0); Cp[c] = C[c * N + p]; }
    om_stress(mat, Fp, s ? s[p] : 1.0, tau);
    for (int c = 0; c < 9; ++c) A[c] = mp * Cp[c] - (4.0 * cfg->dt * V0 / (dx * dx)) * tau[c];
    int out = 0;
    for (int a = 0; a < 3; ++a) {
        double t = x[a * N + p] / dx;
        om_weights(t, &base[a], w[a]);
        f[a] = t - base[a];
        if (base[a] < 0 || base[a] + 2 > n) out = 1;
    }
    return out;
}

/* Add one particle's mass and momentum to its 27 nodes.                    */
static void p2g_scatter(int n, double mp, const double vp[3], const int base[3], double w[3][3],
                        const double f[3], const double A[9], double* gm, double* gp) {
    const double dx = 1.0 / n;
    const long NN = (long)(n + 1) * (n + 1) * (n + 1);
    for (int o0 = 0; o0 < 3; ++o0)
        for (int o1 = 0; o1 < 3; ++o1)
            for (int o2 = 0; o2 < 3; ++o2) {
                double wt = w[0][o0] * w[1][o1] * w[2][o2];
                double d[3] = {(o0 - f[0]) * dx, (o1 - f[1]) * dx, (o2 - f[2]) * dx};
                long id = node_index(n, base[0] + o0, base[1] + o1, base[2] + o2);
                gm[id] += wt * mp;
                for (int a = 0; a < 3; ++a) {
                    double Ad = A[a * 3 + 0] * d[0] + A[a * 3 + 1] * d[1] + A[a * 3 + 2] * d[2];
                    gp[a * NN + id] += wt * (mp * vp[a] + Ad);
                }
            }
}

static double particle_mass(const om_config* cfg, const om_material* mat) {
    const double dx = 1.0 / cfg->n;
    return mat->rho * dx * dx * dx / mat->ppc;
}

long om_p2g(const om_config* cfg, const om_material* mat, long N, const double* x, const double* v,
            const double* C, const double* F, const double* s, double* gm, double* gp) {
    const int n = cfg->n;
    const double mp = particle_mass(cfg, mat);
    const long NN = (long)(n + 1) * (n + 1) * (n + 1);
    memset(gm, 0, sizeof(double) * NN);
    memset(gp, 0, sizeof(double) * 3 * NN);
    long bad = 0;
    for (long p = 0; p < N; ++p) {
        int base[3];
        double w[3][3], f[3], A[9];
        if (p2g_prepare(cfg, mat, N, p, x, C, F, s, base, w, f, A)) { ++bad; continue; }
        double vp[3] = {v[p], v[N + p], v[2 * N + p]};
        p2g_scatter(n, mp, vp, base, w, f, A, gm, gp);
    }
    return bad;
}

/* ------------------------------------------------------------ grid update
 * v_i = p_i / m_i + dt g where m_i > 0, else 0; then the wall condition on
 * every node with a coordinate below bc_cells or above n - bc_cells.
 * Overwrites gp with the nodal velocity.                                    */
static void grid_node(const om_config* cfg, const double* gm, double* gv, int i, int j, int k) {
    const int n = cfg->n, b = cfg->bc_cells;
    const long NN = (long)(n + 1) * (n + 1) * (n + 1);
    long id = node_index(n, i, j, k);
    double vel[3] = {0, 0, 0};
    if (gm[id] > 0.0)
        for (int a = 0; a < 3; ++a) vel[a] = gv[a * NN + id] / gm[id] + cfg->dt * cfg->gravity[a];
    int idx[3] = {i, j, k};
    int lowside[3], highside[3], any = 0;
    for (int a = 0; a < 3; ++a) {
        lowside[a] = idx[a] < b;
        highside[a] = idx[a] > n - b;
        any |= lowside[a] | highside[a];
    }
    if (any) {
        if (cfg->bc == 0) {
            vel[0] = vel[1] = vel[2] = 0.0;
        } else {
            for (int a = 0; a < 3; ++a) {
                if (cfg->bc == 1) {
                    if (lowside[a] || highside[a]) vel[a] = 0.0;
                } else {
                    if (lowside[a] && vel[a] < 0.0) vel[a] = 0.0;
                    if (highside[a] && vel[a] > 0.0) vel[a] = 0.0;
                }
            }
        }
    }
    for (int a = 0; a < 3; ++a) gv[a * NN + id] = vel[a];
}

void om_grid_update(const om_config* cfg, const double* gm, double* gv) {
    const int n = cfg->n;
    for (int i = 0; i <= n; ++i)
        for (int j = 0; j <= n; ++j)
            for (int k = 0; k <= n; ++k) grid_node(cfg, gm, gv, i, j, k);
}

/* -------------------------------------------------------------------- G2P
 * v' = sum w v_i, C' = 4/dx^2 sum w v_i (x_i - x_p)^T, x' = x + dt v',
 * then the material update with the new C'.  In-place on x, v, C, F, s.
 * One particle; returns 1 (and leaves it unchanged) if its stencil leaves
 * the grid.                                                                 */
typedef struct {     /* the ASFLIP transfer (flip = 0: APIC)                          */
    const double* vt; /* [3][(n+1)^3] grid velocity the particles transferred, p_i/m_i  */
    double flip, bmin, bmax;
} om_flip;

static int g2p_particle_map(const om_config* cfg, const om_material* mat, long N, long p, double* x, double* v,
                            double* C, double* F, double* s, const double* gv, int apply_map, const om_flip* fl) {
    const int n = cfg->n;
    const double dx = 1.0 / n, dt = cfg->dt;
    const long NN = (long)(n + 1) * (n + 1) * (n + 1);
    int base[3], out = 0;
    double w[3][3], f[3];
    for (int a = 0; a < 3; ++a) {
        double t = x[a * N + p] / dx;
        om_weights(t, &base[a], w[a]);
        f[a] = t - base[a];
        if (base[a] < 0 || base[a] + 2 > n) out = 1;
    }
    if (out) return 1;
    double vn[3] = {0, 0, 0}, Cn[9] = {0}, vbar[3] = {0, 0, 0};
    for (int o0 = 0; o0 < 3; ++o0)
        for (int o1 = 0; o1 < 3; ++o1)
            for (int o2 = 0; o2 < 3; ++o2) {
                double wt = w[0][o0] * w[1][o1] * w[2][o2];
                double d[3] = {(o0 - f[0]) * dx, (o1 - f[1]) * dx, (o2 - f[2]) * dx};
                long id = node_index(n, base[0] + o0, base[1] + o1, base[2] + o2);
                for (int a = 0; a < 3; ++a) {
                    double vi = gv[a * NN + id];
                    vn[a] += wt * vi;
                    for (int b = 0; b < 3; ++b) Cn[a * 3 + b] += 4.0 / (dx * dx) * wt * vi * d[b];
                    if (fl && fl->flip > 0.0) vbar[a] += wt * fl->vt[a * NN + id];
                }
            }
    double G[9]; /* I + dt C' */
    for (int c = 0; c < 9; ++c) G[c] = dt * Cn[c] + (c % 4 == 0 ? 1.0 : 0.0);
    if (fl && fl->flip > 0.0) {
        /* ASFLIP: v' = v^ + flip (v - v-), x' = x + dt (v^ + beta flip (v - v-)), beta = bmin
         * where the particle's volume is being compressed (J' < 1), bmax elsewhere */
        double J = mat_det(G);
        if (mat->kind == OM_WATER) J *= s[p];
        double beta = J < 1.0 ? fl->bmin : fl->bmax;
        for (int a = 0; a < 3; ++a) {
            double corr = v[a * N + p] - vbar[a];
            x[a * N + p] += dt * (vn[a] + beta * fl->flip * corr);
            v[a * N + p] = vn[a] + fl->flip * corr;
        }
    } else {
        for (int a = 0; a < 3; ++a) {
            v[a * N + p] = vn[a];
            x[a * N + p] += dt * vn[a];
        }
    }
    for (int c = 0; c < 9; ++c) C[c * N + p] = Cn[c];
    if (mat->kind == OM_WATER) {
        s[p] *= mat_det(G);
    } else {
        double Fp[9], Fn[9];
        for (int c = 0; c < 9; ++c) Fp[c] = F[c * N + p];
        mat_mul(G, Fp, Fn);
        if (!apply_map) {
            /* trial gradient only: a caller applies the return map */
        } else if (mat->kind == OM_SNOW) {
            double Fe[9], Jp;
            om_snow_project(mat, Fn, s[p], Fe, &Jp);
            memcpy(Fn, Fe, sizeof Fe);
            s[p] = Jp;
        } else if (mat->kind == OM_SAND) { /* s holds 1 + q */
            double Fe[9], q;
            om_sand_project(mat, Fn, s[p] - 1.0, Fe, &q);
            memcpy(Fn, Fe, sizeof Fe);
            s[p] = 1.0 + q;
        }
        for (int c = 0; c < 9; ++c) F[c * N + p] = Fn[c];
    }
    return 0;
}

static int g2p_particle(const om_config* cfg, const om_material* mat, long N, long p, double* x, double* v,
                        double* C, double* F, double* s, const double* gv) {
    return g2p_particle_map(cfg, mat, N, p, x, v, C, F, s, gv, 1, NULL);
}

long om_g2p(const om_config* cfg, const om_material* mat, long N, double* x, double* v, double* C, double* F,
            double* s, const double* gv) {
    long bad = 0;
    for (long p = 0; p < N; ++p) bad += g2p_particle(cfg, mat, N, p, x, v, C, F, s, gv);
    return bad;
}

/* G2P that stops at the trial gradient F^ = (I + dt C') F (snow, sand: no
 * return map; s unchanged), for a caller that maps F^ itself.              */
long om_g2p_trial(const om_config* cfg, const om_material* mat, long N, double* x, double* v, double* C, double* F,
                  double* s, const double* gv) {
    long bad = 0;
    for (long p = 0; p < N; ++p) bad += g2p_particle_map(cfg, mat, N, p, x, v, C, F, s, gv, 0, NULL);
    return bad;
}

/* One full substep.  gm and gv receive the grid mass and the updated grid
 * velocity of this substep.  Returns the count of out-of-range particles.   */
long om_substep(const om_config* cfg, const om_material* mat, long N, double* x, double* v, double* C, double* F,
                double* s, double* gm, double* gv) {
    long bad = om_p2g(cfg, mat, N, x, v, C, F, s, gm, gv);
    om_grid_update(cfg, gm, gv);
    bad += om_g2p(cfg, mat, N, x, v, C, F, s, gv);
    return bad;
}

/* ------------------------------------------------------------- ASFLIP
 * One substep with the ASFLIP transfer, the integrator the paper's fountain
 * uses (Results, "Fountain"; Fei et al. 2021).  The paper names it without
 * its formulas; the reading here: with v the particle's velocity before the
 * substep, v^ the interpolated new grid velocity and v- the interpolated grid
 * velocity the particles transferred (p_i / m_i, before gravity and walls),
 *   v' = v^ + flip (v - v-),   x' = x + dt (v^ + beta flip (v - v-)),
 * beta = bmin where the particle's volume is being compressed (J' < 1: J
 * det(I + dt C') for water, det(I + dt C') otherwise) and bmax elsewhere; C'
 * and the material update are APIC's.  flip = 0 is the APIC substep.        */
long om_substep_asflip(const om_config* cfg, const om_material* mat, long N, double* x, double* v, double* C,
                       double* F, double* s, double* gm, double* gv, double flip, double bmin, double bmax) {
    const int n = cfg->n;
    const long NN = (long)(n + 1) * (n + 1) * (n + 1);
    long bad = om_p2g(cfg, mat, N, x, v, C, F, s, gm, gv);
    double* vt = malloc(sizeof(double) * 3 * NN);
    for (long i = 0; i < NN; ++i)
        for (int a = 0; a < 3; ++a) vt[a * NN + i] = gm[i] > 0.0 ? gv[a * NN + i] / gm[i] : 0.0;
    om_grid_update(cfg, gm, gv);
    om_flip fl = {vt, flip, bmin, bmax};
    for (long p = 0; p < N; ++p) bad += g2p_particle_map(cfg, mat, N, p, x, v, C, F, s, gv, 1, &fl);
    free(vt);
    return bad;
}

/* ------------------------------------------------ multi-threaded substep
 * The same substep split over OpenMP threads, for timing on many host cores
 * and for long runs in tests.  Particle work (stress, G2P and the material
 * update) is split over particles and the grid update over node planes.
 * P2G keeps one summation order whatever the thread count: the particles
 * are binned, in input order, into slabs of OM_SLAB cells along x by their
 * stencil base; the even slabs scatter first and the odd ones after (inside a
 * slab the particles go in input order; slabs of one parity never share a
 * node, since a slab's stencils span OM_SLAB + 2 nodes).  The result is the
 * single-threaded substep's up to the order of the floating-point sums.
 * threads <= 0 takes the OpenMP default.                                    */
#define OM_SLAB 4
long om_substep_omp(const om_config* cfg, const om_material* mat, long N, double* x, double* v, double* C,
                    double* F, double* s, double* gm, double* gv, int threads) {
    const int n = cfg->n;
    const long NN = (long)(n + 1) * (n + 1) * (n + 1);
    const double mp = particle_mass(cfg, mat);
    const int nslab = n / OM_SLAB + 1;
    if (threads <= 0) threads = omp_get_max_threads();
    int* base = malloc(sizeof(int) * 3 * (N > 0 ? N : 1));
    double* W = malloc(sizeof(double) * 9 * (N > 0 ? N : 1));
    double* fr = malloc(sizeof(double) * 3 * (N > 0 ? N : 1));
    double* A = malloc(sizeof(double) * 9 * (N > 0 ? N : 1));
    long* start = calloc(nslab + 1, sizeof(long));
    long* order = malloc(sizeof(long) * (N > 0 ? N : 1));
    long bad = 0;

#pragma omp parallel for num_threads(threads) schedule(static)
    for (long i = 0; i < NN; ++i) gm[i] = 0.0;
#pragma omp parallel for num_threads(threads) schedule(static)
    for (long i = 0; i < 3 * NN; ++i) gv[i] = 0.0;

#pragma omp parallel for num_threads(threads) schedule(dynamic, 1024) reduction(+ : bad)
    for (long p = 0; p < N; ++p) {
        int b[3];
        double w[3][3];
        int out = p2g_prepare(cfg, mat, N, p, x, C, F, s, b, w, &fr[3 * p], &A[9 * p]);
        for (int a = 0; a < 3; ++a) {
            base[3 * p + a] = out ? -1 : b[a];
            for (int o = 0; o < 3; ++o) W[9 * p + 3 * a + o] = w[a][o];
        }
        bad += out;
    }
    /* stable counting sort of the in-range particles by slab */
    for (long p = 0; p < N; ++p)
        if (base[3 * p] >= 0) start[base[3 * p] / OM_SLAB + 1]++;
    for (int k = 0; k < nslab; ++k) start[k + 1] += start[k];
    {
        long* fill = malloc(sizeof(long) * (nslab > 0 ? nslab : 1));
        memcpy(fill, start, sizeof(long) * nslab);
        for (long p = 0; p < N; ++p)
            if (base[3 * p] >= 0) order[fill[base[3 * p] / OM_SLAB]++] = p;
        free(fill);
    }
    for (int parity = 0; parity < 2; ++parity) {
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1)
        for (int k = parity; k < nslab; k += 2)
            for (long j = start[k]; j < start[k + 1]; ++j) {
                long p = order[j];
                double w[3][3], vp[3] = {v[p], v[N + p], v[2 * N + p]};
                for (int a = 0; a < 3; ++a)
                    for (int o = 0; o < 3; ++o) w[a][o] = W[9 * p + 3 * a + o];
                p2g_scatter(n, mp, vp, &base[3 * p], w, &fr[3 * p], &A[9 * p], gm, gv);
            }
    }
#pragma omp parallel for num_threads(threads) schedule(static)
    for (int i = 0; i <= n; ++i)
        for (int j = 0; j <= n; ++j)
            for (int k = 0; k <= n; ++k) grid_node(cfg, gm, gv, i, j, k);
#pragma omp parallel for num_threads(threads) schedule(dynamic, 1024) reduction(+ : bad)
    for (long p = 0; p < N; ++p) bad += g2p_particle(cfg, mat, N, p, x, v, C, F, s, gv);

    free(base);
    free(W);
    free(fr);
    free(A);
    free(start);
    free(order);
    return bad;
}

/* --------------------------------------------------------------- binning
 * Particle code: c = floor(x/dx + 1/2) = base + 1 per axis (the cell whose
 * centre node is nearest), interleaved bit by bit, x in the lowest bit:
 * code bit 3k = c_x bit k, 3k+1 = c_y bit k, 3k+2 = c_z bit k.  The upper
 * bits are then the block code of c >> 2 and the low six bits the cell code
 * inside the 4^3 block.  Positions are FP32 as stored on the device; the
 * conversion to FP64 is exact.  Returns the number of particles with c
 * outside [1, n-1] (their code uses c clamped into [0, n-1]).               */
long om_keys(long N, const float* x, int n, uint32_t* keys, int32_t* cell) {
    long bad = 0;
    const double dx = 1.0 / n;
    for (long p = 0; p < N; ++p) {
        int c[3], out = 0;
        for (int a = 0; a < 3; ++a) {
            double t = (double)x[a * N + p] / dx;
            double cc = floor(t - 0.5) + 1.0;
            if (!(cc >= 1.0 && cc <= n - 1.0)) out = 1;
            if (!(cc >= 0.0)) cc = 0.0;
            if (cc > n - 1.0) cc = n - 1.0;
            c[a] = (int)cc;
            if (cell) cell[a * N + p] = c[a];
        }
        uint32_t code = 0;
        for (int bit = 0; bit < 10; ++bit)
            for (int a = 0; a < 3; ++a)
                if ((c[a] >> bit) & 1) code |= 1u << (3 * bit + a);
        keys[p] = code;
        bad += out;
    }
    return bad;
}

typedef struct { uint32_t key; long idx; } om_pair;
static int cmp_pair(const void* a, const void* b) {
    const om_pair *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* Stable sort of positions 0..N-1 by key: perm[j] = position of the j-th
 * smallest (ties keep their current order); sorted[j] = keys[perm[j]].      */
void om_stable_sort(long N, const uint32_t* keys, int32_t* perm, uint32_t* sorted) {
    om_pair* t = malloc(sizeof(om_pair) * (N > 0 ? N : 1));
    for (long p = 0; p < N; ++p) { t[p].key = keys[p]; t[p].idx = p; }
    qsort(t, N, sizeof(om_pair), cmp_pair);
    for (long j = 0; j < N; ++j) { perm[j] = (int32_t)t[j].idx; if (sorted) sorted[j] = t[j].key; }
    free(t);
}

/* Geometric blocks from sorted codes: the distinct block codes (code >> 6)
 * in ascending order with their first sorted position and particle count.
 * Returns the number of blocks.                                             */
long om_gblocks(long N, const uint32_t* sorted, uint32_t* bcode, int32_t* start, int32_t* count) {
    long nb = 0;
    for (long j = 0; j < N; ++j) {
        if (j == 0 || (sorted[j] >> 6) != (sorted[j - 1] >> 6)) {
            bcode[nb] = sorted[j] >> 6;
            start[nb] = (int32_t)j;
            count[nb] = 0;
            ++nb;
        }
        count[nb - 1]++;
    }
    return nb;
}

static int unspread(uint32_t code, int a) {
    int v = 0;
    for (int bit = 0; bit < 10; ++bit)
        if ((code >> (3 * bit + a)) & 1) v |= 1 << bit;
    return v;
}

/* Physical blocks: every block within one block (3x3x3) of a geometric
 * block.  Returned as padded linear codes ((bz*NB)+by)*NB+bx with
 * b = blockcoord + 1 and NB = n/4 + 2, ascending.  Returns the count.        */
long om_pblocks(int n, long nb, const uint32_t* bcode, int32_t* out) {
    const int NB = n / 4 + 2;
    const long tot = (long)NB * NB * NB;
    unsigned char* mark = calloc(tot, 1);
    for (long g = 0; g < nb; ++g) {
        int B[3] = {unspread(bcode[g], 0), unspread(bcode[g], 1), unspread(bcode[g], 2)};
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dxx = -1; dxx <= 1; ++dxx) {
                    int bx = B[0] + dxx + 1, by = B[1] + dy + 1, bz = B[2] + dz + 1;
                    mark[((long)bz * NB + by) * NB + bx] = 1;
                }
    }
    long cnt = 0;
    for (long i = 0; i < tot; ++i)
        if (mark[i]) out[cnt++] = (int32_t)i;
    free(mark);
    return cnt;
}

/* Free zone: a particle binned to block B (c >> 2 at the last rebuild) may
 * move while its cell c stays in [4B-3, 4B+6] on every axis: ten cells, so
 * its stencil stays within the 12 nodes of blocks B-1..B+1.  Returns how
 * many particles left it; flags[p] = 1 for those.                            */
long om_free_zone_exit(long N, const float* x, int n, const int32_t* B, uint8_t* flags) {
    const double dx = 1.0 / n;
    long cnt = 0;
    for (long p = 0; p < N; ++p) {
        int out = 0;
        for (int a = 0; a < 3; ++a) {
            double c = floor((double)x[a * N + p] / dx - 0.5) + 1.0;
            double lo = 4.0 * B[a * N + p] - 3.0, hi = 4.0 * B[a * N + p] + 6.0;
            if (c < lo || c > hi) out = 1;
        }
        if (flags) flags[p] = (uint8_t)out;
        cnt += out;
    }
    return cnt;
}
