/*
 * FP64 CPU oracle for the double-distribution-function (DDF) lattice Boltzmann
 * method with local vorticity (Hajabdollahi & Premnath, arXiv:1908.06742).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the GPU
 * library is checked against.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Every arithmetic step follows the paper in its own order and notation:
 *   - D2Q9 velocities and the natural raw-moment basis T        (Sec. 2, eq. particlevelocities, basisvectors)
 *   - m = T f, relaxation in moment space, f* = T^-1 m*         (Sec. 2, eq. MRT-LBEfluidmotion_transformed)
 *   - fluid equilibria and source moments                        (Sec. 2, eq. eqmrawmoment and the sigma' list)
 *   - rho, u with the half-force shift                           (Sec. 2, eq. hydrodynamic_fields)
 *   - scalar MRT with the anisotropic third-order equilibria     (Sec. 3, eq. MRT-LBECDE, eqmrawmoment_CDE)
 *   - local velocity gradient and vorticity                      (Sec. 4, eqs. crossderivativeRHS1/2,
 *                                                                 offdiagvelderivativeresult1/2,
 *                                                                 diagvelderivativeresult1/2, vorticityexpression)
 *   - scalar SRT variant                                         (App. B)
 *   - scalar cascaded central-moment variant                     (App. C)
 *   - scalar non-cascaded central-moment variant                 (App. D)
 * T and its inverse are built from the basis definition and a generic Gauss-Jordan
 * inversion; no hand-derived sparse formula is used.  Streaming is the two-array
 * pull form f(x, n+1) = f*(x - e, n).  Readings where the paper is silent (wall
 * rules, forcing inside the non-equilibrium moments, extraction state) are listed
 * next to the code that applies them.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC ddf_oracle.c -lm
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 9

/* D2Q9 particle velocities in the paper's order (Sec. 2, eq. particlevelocities1/2). */
static const int EX[NQ] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[NQ] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

/* Side indices for wall data: x = -1/2, x = nx - 1/2, y = -1/2, y = ny - 1/2. */
enum { SIDE_LEFT = 0, SIDE_RIGHT = 1, SIDE_BOTTOM = 2, SIDE_TOP = 3 };

/* Scalar collision models. */
enum { SC_MRT = 0, SC_SRT = 1, SC_CASCADED = 2, SC_CENTRAL = 3 };

/* Force kinds. */
enum { FK_NONE = 0, FK_UNIFORM = 1, FK_FOURROLL = 2, FK_PULSATILE = 3 };

typedef struct {
    int nx, ny;
    int periodic_x, periodic_y;     /* 1 = periodic, 0 = half-way walls on both sides */
    double lam_f[NQ];               /* diag(0,0,0,w3..w8) of the fluid MRT (Sec. 2, eq. relaxationtimematrix_fluidmotion) */
    double lam_g[NQ];               /* diag(0,w1..w8) of the scalar MRT (Sec. 3, eq. relaxationtimematrix_CDE) */
    double beta1, beta2;            /* anisotropy of the third-order scalar equilibria */
    double cs2, cs2phi;             /* c_s^2 and c_sphi^2 */
    double wall_ux[4], wall_uy[4];  /* wall velocity per side */
    double wall_phi[4];             /* Dirichlet scalar per side; NaN = zero-flux wall */
    int force_kind;
    double force[2];                /* uniform force, or amplitudes */
    double force_k;                 /* wavenumber of the four-rolls-mill force */
    double force_omega;             /* angular frequency of the pulsatile force */
    int scalar_model;               /* SC_* */
    double phi_min;                 /* |phi| below this: phi-dependent outputs are NaN */
    int nthreads;
} orc_params;

/* ------------------------------------------------------------------------- */
/* Moment algebra                                                             */
/* ------------------------------------------------------------------------- */

/* Natural non-orthogonal basis vector k evaluated at direction a (Sec. 2, eq. basisvectors). */
static double basis_T(int k, int a)
{
    const double x = EX[a], y = EY[a];
    switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return x * x + y * y;
    case 4: return x * x - y * y;
    case 5: return x * y;
    case 6: return x * x * y;
    case 7: return x * y * y;
    default: return x * x * y * y;
    }
}

/* Bare raw-moment basis P (App. B, eq. basisvectors1). */
static double basis_P(int k, int a)
{
    const double x = EX[a], y = EY[a];
    switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return x * x;
    case 4: return y * y;
    case 5: return x * y;
    case 6: return x * x * y;
    case 7: return x * y * y;
    default: return x * x * y * y;
    }
}

/* Generic Gauss-Jordan inverse with partial pivoting of an n x n row-major matrix.
 * Returns 0 on success, -1 if singular. */
static int invert(int n, const double *A, double *Ainv)
{
    double M[NQ][2 * NQ];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < 2 * n; ++j)
            M[i][j] = (j < n) ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (fabs(M[r][c]) > fabs(M[p][c])) p = r;
        if (fabs(M[p][c]) < 1e-300) return -1;
        if (p != c)
            for (int j = 0; j < 2 * n; ++j) { double t = M[c][j]; M[c][j] = M[p][j]; M[p][j] = t; }
        const double d = M[c][c];
        for (int j = 0; j < 2 * n; ++j) M[c][j] /= d;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double s = M[r][c];
            if (s != 0.0)
                for (int j = 0; j < 2 * n; ++j) M[r][j] -= s * M[c][j];
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Ainv[i * n + j] = M[i][j + n];
    return 0;
}

static double T_[NQ * NQ], Tinv_[NQ * NQ], P_[NQ * NQ], Pinv_[NQ * NQ];
static int algebra_ready = 0;

static void ensure_algebra(void)
{
    if (algebra_ready) return;
    for (int k = 0; k < NQ; ++k)
        for (int a = 0; a < NQ; ++a) {
            T_[k * NQ + a] = basis_T(k, a);
            P_[k * NQ + a] = basis_P(k, a);
        }
    invert(NQ, T_, Tinv_);
    invert(NQ, P_, Pinv_);
    algebra_ready = 1;
}

static void matvec(const double *A, const double *v, double *out)
{
    for (int i = 0; i < NQ; ++i) {
        double s = 0.0;
        for (int j = 0; j < NQ; ++j) s += A[i * NQ + j] * v[j];
        out[i] = s;
    }
}

/* Exported for tests: T, T^-1, P, P^-1 (row-major 9x9). */
void orc_matrices(double *T, double *Tinv, double *P, double *Pinv)
{
    ensure_algebra();
    memcpy(T, T_, sizeof T_);
    memcpy(Tinv, Tinv_, sizeof Tinv_);
    memcpy(P, P_, sizeof P_);
    memcpy(Pinv, Pinv_, sizeof Pinv_);
}

/* ------------------------------------------------------------------------- */
/* Equilibria and source (Sec. 2 and Sec. 3)                                 */
/* ------------------------------------------------------------------------- */

/* Raw-moment fluid equilibria (Sec. 2, eq. eqmrawmoment) in the T-ordering
 * (kappa_0, kappa_x, kappa_y, kappa_xx+kappa_yy, kappa_xx-kappa_yy, kappa_xy,
 *  kappa_xxy, kappa_xyy, kappa_xxyy). */
void orc_meq_fluid(double rho, double ux, double uy, double cs2, double *meq)
{
    const double kxx = cs2 * rho + rho * ux * ux;
    const double kyy = cs2 * rho + rho * uy * uy;
    meq[0] = rho;
    meq[1] = rho * ux;
    meq[2] = rho * uy;
    meq[3] = kxx + kyy;
    meq[4] = kxx - kyy;
    meq[5] = rho * ux * uy;
    meq[6] = cs2 * rho * uy + rho * ux * ux * uy;
    meq[7] = cs2 * rho * ux + rho * ux * uy * uy;
    meq[8] = cs2 * cs2 * rho + cs2 * rho * (ux * ux + uy * uy) + rho * ux * ux * uy * uy;
}

/* Raw-moment scalar equilibria with the anisotropic third-order terms
 * (Sec. 3, eq. eqmrawmoment_CDE), in the T-ordering. */
void orc_neq_scalar(double phi, double ux, double uy, double cs2p, double b1, double b2, double *neq)
{
    const double exx = cs2p * phi + phi * ux * ux;
    const double eyy = cs2p * phi + phi * uy * uy;
    neq[0] = phi;
    neq[1] = phi * ux;
    neq[2] = phi * uy;
    neq[3] = exx + eyy;
    neq[4] = exx - eyy;
    neq[5] = phi * ux * uy;
    neq[6] = b1 * cs2p * phi * uy + phi * ux * ux * uy;
    neq[7] = b2 * cs2p * phi * ux + phi * ux * uy * uy;
    neq[8] = cs2p * cs2p * phi + cs2p * phi * (ux * ux + uy * uy) + phi * ux * ux * uy * uy;
}

/* Same scalar equilibria in the bare ordering of App. B (eq. momentequilibriaCDE1). */
static void qeq_scalar_bare(double phi, double ux, double uy, double cs2p, double b1, double b2, double *q)
{
    q[0] = phi;
    q[1] = phi * ux;
    q[2] = phi * uy;
    q[3] = cs2p * phi + phi * ux * ux;
    q[4] = cs2p * phi + phi * uy * uy;
    q[5] = phi * ux * uy;
    q[6] = b1 * cs2p * phi * uy + phi * ux * ux * uy;
    q[7] = b2 * cs2p * phi * ux + phi * ux * uy * uy;
    q[8] = cs2p * cs2p * phi + cs2p * phi * (ux * ux + uy * uy) + phi * ux * ux * uy * uy;
}

/* Raw moments of the source term (Sec. 2, the sigma' list), T-ordering. */
void orc_source_moments(double Fx, double Fy, double ux, double uy, double *S)
{
    const double sxx = 2.0 * Fx * ux;
    const double syy = 2.0 * Fy * uy;
    S[0] = 0.0;
    S[1] = Fx;
    S[2] = Fy;
    S[3] = sxx + syy;
    S[4] = sxx - syy;
    S[5] = Fx * uy + Fy * ux;
    S[6] = Fy * ux * ux + 2.0 * Fx * ux * uy;
    S[7] = Fx * uy * uy + 2.0 * Fy * uy * ux;
    S[8] = 2.0 * (Fx * ux * uy * uy + Fy * uy * ux * ux);
}

/* Body force at node (i, j) and time t. */
static void force_at(const orc_params *p, int i, int j, double t, double *Fx, double *Fy)
{
    switch (p->force_kind) {
    case FK_UNIFORM:
        *Fx = p->force[0]; *Fy = p->force[1];
        break;
    case FK_FOURROLL: {
        /* four-rolls mill (Sec. 5.2): F = F0 (sin x sin y, cos x cos y), x = k i */
        const double x = p->force_k * i, y = p->force_k * j;
        *Fx = p->force[0] * sin(x) * sin(y);
        *Fy = p->force[0] * cos(x) * cos(y);
        break;
    }
    case FK_PULSATILE: {
        /* Womersley (Sec. 5.3): F_x = F_m cos(Omega t) */
        const double c = cos(p->force_omega * t);
        *Fx = p->force[0] * c; *Fy = p->force[1] * c;
        break;
    }
    default:
        *Fx = 0.0; *Fy = 0.0;
    }
}

/* Equilibrium populations T^-1 m_eq (used for initialisation and walls). */
static void feq_fluid(double rho, double ux, double uy, double cs2, double *feq)
{
    double m[NQ];
    orc_meq_fluid(rho, ux, uy, cs2, m);
    matvec(Tinv_, m, feq);
}

static void geq_scalar(double phi, double ux, double uy, const orc_params *p, double *geq)
{
    double n[NQ];
    orc_neq_scalar(phi, ux, uy, p->cs2phi, p->beta1, p->beta2, n);
    matvec(Tinv_, n, geq);
}

/* ------------------------------------------------------------------------- */
/* Scalar collision variants                                                  */
/* ------------------------------------------------------------------------- */

/* Sec. 3, eq. MRT-LBECDE: g* = g - T^-1 [Lambda^phi (n - n_eq)]. */
static void collide_scalar_mrt(const orc_params *p, const double *g, double phi, double ux, double uy, double *gs)
{
    double n[NQ], neq[NQ], ns[NQ];
    matvec(T_, g, n);
    orc_neq_scalar(phi, ux, uy, p->cs2phi, p->beta1, p->beta2, neq);
    for (int k = 0; k < NQ; ++k) ns[k] = n[k] - p->lam_g[k] * (n[k] - neq[k]);
    matvec(Tinv_, ns, gs);
}

/* App. B: SRT with g_eq = P^-1 q_eq and rate 1/tau_phi = lam_g[1]. */
static void collide_scalar_srt(const orc_params *p, const double *g, double phi, double ux, double uy, double *gs)
{
    double q[NQ], geq[NQ];
    qeq_scalar_bare(phi, ux, uy, p->cs2phi, p->beta1, p->beta2, q);
    matvec(Pinv_, q, geq);
    const double w = p->lam_g[1];
    for (int a = 0; a < NQ; ++a) gs[a] = g[a] - w * (g[a] - geq[a]);
}

/* Central moment (m, n) of a population vector about u, by its definition (App. C, eq. centralmomentdefinitions_CDE). */
static double central_moment(const double *g, int m, int n, double ux, double uy)
{
    double s = 0.0;
    for (int a = 0; a < NQ; ++a) s += g[a] * pow(EX[a] - ux, m) * pow(EY[a] - uy, n);
    return s;
}

/* Central-moment equilibria with the boxed anisotropic third-order terms (App. C, eq. eqmcentralmoment_CDE).
 * Order: 0, x, y, xx, yy, xy, xxy, xyy, xxyy. */
static void cm_eq(double phi, double ux, double uy, const orc_params *p, double *c)
{
    const double cs2 = p->cs2phi;
    c[0] = phi;
    c[1] = 0.0;
    c[2] = 0.0;
    c[3] = cs2 * phi;
    c[4] = cs2 * phi;
    c[5] = 0.0;
    c[6] = (p->beta1 - 1.0) * cs2 * phi * uy;
    c[7] = (p->beta2 - 1.0) * cs2 * phi * ux;
    c[8] = cs2 * cs2 * phi;
}

static const int CM_M[NQ] = {0, 1, 0, 2, 0, 1, 2, 1, 2};
static const int CM_N[NQ] = {0, 0, 1, 0, 2, 1, 1, 2, 2};

/* Orthogonal basis of App. C (eq. orthogonalbasisvectors) as K[a*9 + k] = K_k(e_a).
 * The printed K6, K7 lack their lower-order parts; the inner products
 * (eq. innerproductscollisionchanges) and the printed population updates both
 * require K6 = 2|e_y> - 3|e_x^2 e_y> and K7 = 2|e_x> - 3|e_x e_y^2>, which are
 * also the only such choices orthogonal to K2 and K1. */
void orc_cascaded_basis(double *K)
{
    for (int a = 0; a < NQ; ++a) {
        const double x = EX[a], y = EY[a];
        const double row[NQ] = {1.0, x, y, 3.0 * (x * x + y * y) - 4.0, x * x - y * y, x * y,
                                2.0 * y - 3.0 * x * x * y, 2.0 * x - 3.0 * x * y * y,
                                9.0 * x * x * y * y - 6.0 * (x * x + y * y) + 4.0};
        for (int k = 0; k < NQ; ++k) K[a * NQ + k] = row[k];
    }
}

/* App. C: cascaded collision.  The changes h are taken in the paper's cascade
 * order (each uses the lower-order ones) and applied through the orthogonal
 * basis K (eq. orthogonalbasisvectors). */
static void collide_scalar_cascaded(const orc_params *p, const double *g, double ux, double uy, double *gs)
{
    double c[NQ], ce[NQ], h[NQ];
    for (int k = 0; k < NQ; ++k) c[k] = central_moment(g, CM_M[k], CM_N[k], ux, uy);
    cm_eq(c[0], ux, uy, p, ce);
    const double *w = p->lam_g; /* w[1]..w[8] */
    h[0] = 0.0;
    h[1] = w[1] / 6.0 * (ce[1] - c[1]);
    h[2] = w[2] / 6.0 * (ce[2] - c[2]);
    h[3] = w[3] / 12.0 * ((ce[3] + ce[4]) - (c[3] + c[4])) + (ux * h[1] + uy * h[2]);
    h[4] = w[4] / 4.0 * ((ce[3] - ce[4]) - (c[3] - c[4])) + 3.0 * (ux * h[1] - uy * h[2]);
    h[5] = w[5] / 4.0 * (ce[5] - c[5]) + 1.5 * (ux * h[2] + uy * h[1]);
    h[6] = -w[6] / 4.0 * (ce[6] - c[6]) - 2.0 * ux * h[5] - 0.5 * uy * h[4] - 1.5 * uy * h[3]
           + (1.0 + 1.5 * ux * ux) * h[2] + 3.0 * ux * uy * h[1];
    h[7] = -w[7] / 4.0 * (ce[7] - c[7]) - 2.0 * uy * h[5] + 0.5 * ux * h[4] - 1.5 * ux * h[3]
           + 3.0 * ux * uy * h[2] + (1.0 + 1.5 * uy * uy) * h[1];
    h[8] = w[8] / 4.0 * (ce[8] - c[8]) - 2.0 * ux * h[7] - 2.0 * uy * h[6] - 4.0 * ux * uy * h[5]
           + 0.5 * (ux * ux - uy * uy) * h[4] - (2.0 + 1.5 * (ux * ux + uy * uy)) * h[3]
           + (2.0 + 3.0 * ux * ux) * uy * h[2] + (2.0 + 3.0 * uy * uy) * ux * h[1];
    double K[NQ * NQ];
    orc_cascaded_basis(K);
    for (int a = 0; a < NQ; ++a) {
        double s = 0.0;
        for (int k = 0; k < NQ; ++k) s += K[a * NQ + k] * h[k];
        gs[a] = g[a] + s;
    }
}

/* App. D: non-cascaded central-moment collision.  Pre-collision central moments
 * by definition, relaxation of (x, y, xx+yy, xx-yy, xy, xxy, xyy, xxyy), and
 * post-collision populations by solving C(u) g* = c* with the same generic
 * elimination (C(u) holds the central basis vectors at u). */
static void collide_scalar_central(const orc_params *p, const double *g, double ux, double uy, double *gs)
{
    double c[NQ], ce[NQ], cs[NQ];
    for (int k = 0; k < NQ; ++k) c[k] = central_moment(g, CM_M[k], CM_N[k], ux, uy);
    cm_eq(c[0], ux, uy, p, ce);
    const double *w = p->lam_g;
    cs[0] = c[0];
    cs[1] = c[1] + w[1] * (ce[1] - c[1]);
    cs[2] = c[2] + w[2] * (ce[2] - c[2]);
    const double sp = (c[3] + c[4]) + w[3] * ((ce[3] + ce[4]) - (c[3] + c[4]));
    const double sm = (c[3] - c[4]) + w[4] * ((ce[3] - ce[4]) - (c[3] - c[4]));
    cs[3] = 0.5 * (sp + sm);
    cs[4] = 0.5 * (sp - sm);
    cs[5] = c[5] + w[5] * (ce[5] - c[5]);
    cs[6] = c[6] + w[6] * (ce[6] - c[6]);
    cs[7] = c[7] + w[7] * (ce[7] - c[7]);
    cs[8] = c[8] + w[8] * (ce[8] - c[8]);
    double C[NQ * NQ], Ci[NQ * NQ];
    for (int k = 0; k < NQ; ++k)
        for (int a = 0; a < NQ; ++a)
            C[k * NQ + a] = pow(EX[a] - ux, CM_M[k]) * pow(EY[a] - uy, CM_N[k]);
    invert(NQ, C, Ci);
    matvec(Ci, cs, gs);
}

/* ------------------------------------------------------------------------- */
/* One node: macroscopic fields and collision                                 */
/* ------------------------------------------------------------------------- */

/* rho, u (with half force), phi from pre-collision populations (Sec. 2, eq. hydrodynamic_fields; Sec. 3). */
static void macros(const orc_params *p, const double *f, const double *g, double Fx, double Fy,
                   double *rho, double *ux, double *uy, double *phi, double *m, double *n)
{
    (void)p;
    matvec(T_, f, m);
    matvec(T_, g, n);
    *rho = m[0];
    *ux = (m[1] + 0.5 * Fx) / m[0];
    *uy = (m[2] + 0.5 * Fy) / m[0];
    *phi = n[0];
}

/* Fluid collision (Sec. 2, eq. MRT-LBEfluidmotion_transformed):
 * m* = m - Lambda (m - m_eq) + (I - Lambda/2) S;  f* = T^-1 m*. */
static void collide_fluid(const orc_params *p, const double *m, double rho, double ux, double uy,
                          double Fx, double Fy, double *fs)
{
    double meq[NQ], S[NQ], ms[NQ];
    orc_meq_fluid(rho, ux, uy, p->cs2, meq);
    orc_source_moments(Fx, Fy, ux, uy, S);
    for (int k = 0; k < NQ; ++k)
        ms[k] = m[k] - p->lam_f[k] * (m[k] - meq[k]) + (1.0 - 0.5 * p->lam_f[k]) * S[k];
    matvec(Tinv_, ms, fs);
}

static void collide_scalar(const orc_params *p, const double *g, double phi, double ux, double uy, double *gs)
{
    switch (p->scalar_model) {
    case SC_SRT: collide_scalar_srt(p, g, phi, ux, uy, gs); break;
    case SC_CASCADED: collide_scalar_cascaded(p, g, ux, uy, gs); break;
    case SC_CENTRAL: collide_scalar_central(p, g, ux, uy, gs); break;
    default: collide_scalar_mrt(p, g, phi, ux, uy, gs);
    }
}

/* Exported for tests: one collision of a single node (populations in velocity space). */
void orc_collide_node(const orc_params *p, const double *f, const double *g, double Fx, double Fy,
                      double *fs, double *gs)
{
    ensure_algebra();
    double rho, ux, uy, phi, m[NQ], n[NQ];
    macros(p, f, g, Fx, Fy, &rho, &ux, &uy, &phi, m, n);
    collide_fluid(p, m, rho, ux, uy, Fx, Fy, fs);
    collide_scalar(p, g, phi, ux, uy, gs);
}

/* ------------------------------------------------------------------------- */
/* Lattice                                                                    */
/* ------------------------------------------------------------------------- */

#define IDX(p, a, i, j) ((size_t)(a) * (size_t)(p)->nx * (size_t)(p)->ny + (size_t)(j) * (size_t)(p)->nx + (size_t)(i))

static int opposite(int a)
{
    for (int b = 0; b < NQ; ++b)
        if (EX[b] == -EX[a] && EY[b] == -EY[a]) return b;
    return a;
}

/* Equilibrium initial state from (rho, u, phi) planes (ny x nx each):
 * f_bar = T^-1 (m_eq - S/2) so that u recovered with the half-force shift equals u,
 * and g = T^-1 n_eq. */
void orc_init(const orc_params *p, const double *rho, const double *ux, const double *uy,
              const double *phi, double *f, double *g)
{
    ensure_algebra();
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            const size_t c = (size_t)j * p->nx + i;
            double Fx, Fy, meq[NQ], S[NQ], mb[NQ], fv[NQ], gv[NQ];
            force_at(p, i, j, 0.0, &Fx, &Fy);
            orc_meq_fluid(rho[c], ux[c], uy[c], p->cs2, meq);
            orc_source_moments(Fx, Fy, ux[c], uy[c], S);
            for (int k = 0; k < NQ; ++k) mb[k] = meq[k] - 0.5 * S[k];
            matvec(Tinv_, mb, fv);
            geq_scalar(phi[c], ux[c], uy[c], p, gv);
            for (int a = 0; a < NQ; ++a) {
                f[IDX(p, a, i, j)] = fv[a];
                g[IDX(p, a, i, j)] = gv[a];
            }
        }
}

/* Which wall a link from node (i, j) to (i + dx, j + dy) crosses, or -1 if the
 * target is a fluid node (after periodic wrapping).  A diagonal link leaving
 * through a corner is charged to the bottom or top wall, so that every link a
 * node sends through a moving lid carries the lid velocity (this keeps the
 * momentum-augmentation terms of one node summing to zero mass). */
static int wall_of_link(const orc_params *p, int i, int j, int dx, int dy, int *ti, int *tj)
{
    int x = i + dx, y = j + dy;
    if (p->periodic_x) x = (x + p->nx) % p->nx;
    if (p->periodic_y) y = (y + p->ny) % p->ny;
    *ti = x; *tj = y;
    if (y < 0) return SIDE_BOTTOM;
    if (y >= p->ny) return SIDE_TOP;
    if (x < 0) return SIDE_LEFT;
    if (x >= p->nx) return SIDE_RIGHT;
    return -1;
}

/* Advance nsteps from time t0.  f, g hold the state (9 planes of ny x nx each).
 * Collision of every node into separate post-collision arrays, then pull
 * streaming.  Walls (reading of the half-way rules the paper cites):
 *   fluid:  f_a(x, n+1) = f*_abar(x, n) - [f_eq_abar(rho(x,n), u_w) - f_eq_a(rho(x,n), u_w)]
 *   scalar: g_a(x, n+1) = -g*_abar(x, n) + [g_eq_abar(phi_w, u_w) + g_eq_a(phi_w, u_w)]   (Dirichlet)
 *           g_a(x, n+1) =  g*_abar(x, n)                                            (zero flux, phi_w = NaN)
 * where abar is the direction that left x towards the wall. */
int orc_step(const orc_params *p, double *f, double *g, long nsteps, long t0)
{
    ensure_algebra();
    const size_t N = (size_t)p->nx * p->ny;
    double *fs = (double *)malloc(sizeof(double) * NQ * N);
    double *gs = (double *)malloc(sizeof(double) * NQ * N);
    double *rh = (double *)malloc(sizeof(double) * N);
    if (!fs || !gs || !rh) { free(fs); free(gs); free(rh); return -1; }
#ifdef _OPENMP
    if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#endif
    int opp[NQ];
    for (int a = 0; a < NQ; ++a) opp[a] = opposite(a);

    for (long s = 0; s < nsteps; ++s) {
        const double t = (double)(t0 + s);
        /* collision */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                double fv[NQ], gv[NQ], fo[NQ], go[NQ], Fx, Fy;
                for (int a = 0; a < NQ; ++a) { fv[a] = f[IDX(p, a, i, j)]; gv[a] = g[IDX(p, a, i, j)]; }
                force_at(p, i, j, t, &Fx, &Fy);
                double rho, ux, uy, phi, m[NQ], n[NQ];
                macros(p, fv, gv, Fx, Fy, &rho, &ux, &uy, &phi, m, n);
                collide_fluid(p, m, rho, ux, uy, Fx, Fy, fo);
                collide_scalar(p, gv, phi, ux, uy, go);
                for (int a = 0; a < NQ; ++a) { fs[IDX(p, a, i, j)] = fo[a]; gs[IDX(p, a, i, j)] = go[a]; }
                rh[(size_t)j * p->nx + i] = rho;
            }
        /* pull streaming with walls */
#pragma omp parallel for schedule(static)
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                for (int a = 0; a < NQ; ++a) {
                    int si, sj;
                    const int w = wall_of_link(p, i, j, -EX[a], -EY[a], &si, &sj);
                    if (w < 0) {
                        f[IDX(p, a, i, j)] = fs[IDX(p, a, si, sj)];
                        g[IDX(p, a, i, j)] = gs[IDX(p, a, si, sj)];
                    } else {
                        const int b = opp[a]; /* left x towards the wall */
                        double fe[NQ], ge[NQ];
                        feq_fluid(rh[(size_t)j * p->nx + i], p->wall_ux[w], p->wall_uy[w], p->cs2, fe);
                        f[IDX(p, a, i, j)] = fs[IDX(p, b, i, j)] - (fe[b] - fe[a]);
                        if (isnan(p->wall_phi[w])) {
                            g[IDX(p, a, i, j)] = gs[IDX(p, b, i, j)];
                        } else {
                            geq_scalar(p->wall_phi[w], p->wall_ux[w], p->wall_uy[w], p, ge);
                            g[IDX(p, a, i, j)] = -gs[IDX(p, b, i, j)] + (ge[b] + ge[a]);
                        }
                    }
                }
            }
    }
    free(fs); free(gs); free(rh);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Local kinematics (Sec. 4)                                                  */
/* ------------------------------------------------------------------------- */

enum {
    OUT_RHO = 0, OUT_UX, OUT_UY, OUT_PHI, OUT_SXX, OUT_SYY, OUT_SXY, OUT_WZ,
    OUT_DXUY, OUT_DYUX, OUT_DXPHI, OUT_DYPHI, OUT_Q, OUT_R, OUT_LX, OUT_LY, OUT_N
};

/* Velocity gradient, vorticity and scalar gradient of one node from its
 * pre-collision populations (the state at time t).  Non-equilibrium moments are
 * taken as m - m_eq + S/2 for the fluid, because the scheme evolves
 * f_bar = f - S/2 while the Chapman-Enskog relations hold for f. */
void orc_extract_node(const orc_params *p, const double *f, const double *g, double Fx, double Fy, double *o)
{
    ensure_algebra();
    double rho, ux, uy, phi, m[NQ], n[NQ], meq[NQ], S[NQ], neq[NQ];
    macros(p, f, g, Fx, Fy, &rho, &ux, &uy, &phi, m, n);
    orc_meq_fluid(rho, ux, uy, p->cs2, meq);
    orc_source_moments(Fx, Fy, ux, uy, S);
    orc_neq_scalar(phi, ux, uy, p->cs2phi, p->beta1, p->beta2, neq);
    const double cs2 = p->cs2, cp2 = p->cs2phi, b1 = p->beta1, b2 = p->beta2;
    const double w3 = p->lam_f[3], w4 = p->lam_f[4], w5 = p->lam_f[5];
    const double w1p = p->lam_g[1], w2p = p->lam_g[2], w5p = p->lam_g[5];

    /* second-order non-equilibrium fluid moments (Sec. 4) */
    const double m3 = m[3] - meq[3] + 0.5 * S[3];
    const double m4 = m[4] - meq[4] + 0.5 * S[4];
    const double m5 = m[5] - meq[5] + 0.5 * S[5];
    /* diagonal gradients (eqs. diagvelderivativeresult1/2) */
    const double dxux = -(w3 * m3 + w4 * m4) / (4.0 * cs2 * rho);
    const double dyuy = -(w3 * m3 - w4 * m4) / (4.0 * cs2 * rho);
    /* N_xy (eq. crossderivativeRHS1) */
    const double Nxy = -w5 * m5 / (rho * cs2);
    /* scalar gradient from the first-order non-equilibrium moments (eqs. 1stnoneqmmomentx/y_CDE) */
    const double dxphi = -(w1p / cp2) * (n[1] - neq[1]);
    const double dyphi = -(w2p / cp2) * (n[2] - neq[2]);
    /* N^phi_xy (eq. crossderivativeRHS2).  The central-moment schemes (App. C, D)
     * relax the central moment eta_xy = n5 - u_y n1 - u_x n2 + u_x u_y phi instead of
     * n5; redoing the first-order Chapman-Enskog step of Sec. 3.1 for that moment gives
     * eta_xy^(1) = -(c^2/w5)[phi(b1 dxuy + b2 dyux) + (b1-1) u_y dxphi + (b2-1) u_x dyphi]. */
    double Nphi;
    if (p->scalar_model == SC_CASCADED || p->scalar_model == SC_CENTRAL) {
        const double c5 = central_moment(g, 1, 1, ux, uy);
        Nphi = -w5p * c5 / (phi * cp2) - ((b1 - 1.0) * uy * dxphi + (b2 - 1.0) * ux * dyphi) / phi;
    } else {
        const double n5 = n[5] - neq[5];
        Nphi = -w5p * n5 / (phi * cp2) - (b1 * uy * dxphi + b2 * ux * dyphi) / phi;
    }
    /* cross derivatives and vorticity (eqs. offdiagvelderivativeresult1/2, vorticityexpression) */
    double dxuy = (Nphi - b2 * Nxy) / (b1 - b2);
    double dyux = (b1 * Nxy - Nphi) / (b1 - b2);
    double wz = (2.0 * Nphi - (b1 + b2) * Nxy) / (b1 - b2);
    if (!(fabs(phi) >= p->phi_min)) { dxuy = NAN; dyux = NAN; wz = NAN; }

    const double Sxx = dxux, Syy = dyuy, Sxy = 0.5 * Nxy;
    o[OUT_RHO] = rho; o[OUT_UX] = ux; o[OUT_UY] = uy; o[OUT_PHI] = phi;
    o[OUT_SXX] = Sxx; o[OUT_SYY] = Syy; o[OUT_SXY] = Sxy; o[OUT_WZ] = wz;
    o[OUT_DXUY] = dxuy; o[OUT_DYUX] = dyux; o[OUT_DXPHI] = dxphi; o[OUT_DYPHI] = dyphi;
    /* invariants and Lamb vector of Sec. 1 for a planar flow (omega = (0, 0, wz), S_zz = 0) */
    const double SS = Sxx * Sxx + Syy * Syy + 2.0 * Sxy * Sxy;
    o[OUT_Q] = -0.5 * SS + 0.25 * wz * wz;
    double S3 = 0.0; /* S_ij S_jk S_ki over the 2x2 block */
    {
        const double A[2][2] = {{Sxx, Sxy}, {Sxy, Syy}};
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int k = 0; k < 2; ++k) S3 += A[i][j] * A[j][k] * A[k][i];
    }
    o[OUT_R] = S3 / 3.0; /* the omega_i omega_j S_ij term vanishes: only omega_z, S_zz = 0 */
    /* L = omega x u with omega = (0, 0, wz) */
    o[OUT_LX] = -wz * uy;
    o[OUT_LY] = wz * ux;
}

/* Extraction over the lattice: out holds OUT_N planes of ny x nx. */
void orc_extract(const orc_params *p, const double *f, const double *g, long t, double *out)
{
    ensure_algebra();
    const size_t N = (size_t)p->nx * p->ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            double fv[NQ], gv[NQ], o[OUT_N], Fx, Fy;
            for (int a = 0; a < NQ; ++a) { fv[a] = f[IDX(p, a, i, j)]; gv[a] = g[IDX(p, a, i, j)]; }
            force_at(p, i, j, (double)t, &Fx, &Fy);
            orc_extract_node(p, fv, gv, Fx, Fy, o);
            for (int k = 0; k < OUT_N; ++k) out[(size_t)k * N + (size_t)j * p->nx + i] = o[k];
        }
}

/* Exported: body force at a node (tests use it to build exact source terms). */
void orc_force(const orc_params *p, int i, int j, double t, double *F)
{
    force_at(p, i, j, t, &F[0], &F[1]);
}

int orc_num_outputs(void) { return OUT_N; }
int orc_sizeof_params(void) { return (int)sizeof(orc_params); }
