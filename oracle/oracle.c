/*
 * FP64 CPU oracle for the FDTD-PIC time step of Liu, Zhao, Wang & Liu,
 * "Numerical study of three-dimensional PIC for the surface plasmon
 * excitation based on Drude model" (arXiv:1505.04007).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * code, header or constant table with the GPU library.
 *
 * Everything is SI and double precision.  Each Yee component is stored with
 * its own extents on the full staggered lattice (Sec. II, the index
 * convention stated after Eq. 6):
 *   Ex[nx][ny+1][nz+1] at (i+1/2, j, k)    Hx[nx+1][ny][nz] at (i, j+1/2, k+1/2)
 *   Ey[nx+1][ny][nz+1] at (i, j+1/2, k)    Hy[nx][ny+1][nz] at (i+1/2, j, k+1/2)
 *   Ez[nx+1][ny+1][nz] at (i, j, k+1/2)    Hz[nx][ny][nz+1] at (i+1/2, j+1/2, k)
 * C order, k fastest.  On a periodic axis node n duplicates node 0 and is
 * re-synchronised after every E update.
 *
 * One step n -> n+1 (Sec. II, text after Eq. 8: polarization current first,
 * then E; magnetic field as in vacuum; particles through the Yee fields):
 *   1. H^{n+1/2} = H^{n-1/2} - (dt/mu0) curl E^n                 (vacuum form)
 *   2. particles: gather E^n, B^n = mu0 (H^{n-1/2} + H^{n+1/2}) / 2,
 *      relativistic Boris push, move, Esirkepov deposit of J_b^{n+1/2}
 *   3. J^{n+1/2} = ca J^{n-1/2} + cb E^n on every E edge           (Eq. 6)
 *   4. E^{n+1} = E^n + (dt/eps0)(curl H^{n+1/2} - J^{n+1/2} - J_b^{n+1/2})
 *                                                                  (Eq. 8)
 *   5. probes: F_p(w) += dt Ez_p^{n+1} exp(-i w (n+1) dt)
 * with ca = (2 - g dt)/(2 + g dt), cb = 2 dt eps0 wp^2/(2 + g dt) (Eq. 6).
 * Readings where the paper is silent or garbled (E^n in Eq. 6, the lost
 * minus sign of Eq. 8, beam current in Eq. 8, pusher/deposit scheme, CPML
 * in place of the split-field PML, edge material rule) are the ones listed
 * in the design notes; each is restated at the code that applies it.
 *
 * Pins: every part is checked against closed forms, exact invariants or brute
 * force in the test suite.  The CPML layers are held to the z-domain
 * dispersion roots of a uniformly stretched periodic axis (the psi recursion
 * and its 1/kappa), to the conserved kappa-weighted Yee energy of graded
 * lossless layers (which node or half node each coefficient belongs to), and
 * to the recursive convolution of the continuous CPML kernel (b and c from
 * sigma, kappa, alpha); the grading polynomial itself is a chosen reading.
 * The osim_test_* entries exist for those pins only.
 *
 * The differentiable form (the gradient of probe spectral power with respect
 * to the per-cell wp and gamma of Eq. 1) is the plain reverse-time transpose
 * of steps 1, 3 and 4 with the bunch current of step 2 held at the values a
 * forward run produced; it is written at the end of this file.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_C 299792458.0
#define OR_MU0 1.25663706212e-6
#define OR_EPS0 (1.0 / (OR_MU0 * OR_C * OR_C))
#define OR_ETA0 (OR_MU0 * OR_C)

enum { OR_PEC = 0, OR_PERIODIC = 1, OR_CPML = 2 };

typedef struct {
    int n[3];
    double *v;
} ofield;

#define AT(f, i, j, k) \
    ((f).v[((size_t)(i) * (size_t)(f).n[1] + (size_t)(j)) * (size_t)(f).n[2] + (size_t)(k)])

typedef struct {
    int n[3];
    int bc[3];
    int npml;
    double dx, dt;
    ofield E[3], H[3], Hprev[3], J[3], P[3], Jb[3], ca[3], cb[3];
    /* psiE[c][a]: CPML memory of E component c for its derivative along a */
    ofield psiE[3][3], psiH[3][3];
    /* CPML profile along each axis: E-type at nodes 0..n, H-type at i+1/2 */
    double *bE[3], *cE[3], *kE[3], *bH[3], *cH[3], *kH[3];
    unsigned char *lE[3], *lH[3];
    /* particles */
    long np;
    double *x, *y, *z, *ux, *uy, *uz;
    unsigned char *alive;
    double q, m, w;
    /* probes */
    int nprobe, nfreq;
    int *pijk;
    double *omega, *fre, *fim;
    long step;
    double t_field, t_part;
    long pushes;
    /* bunch current as a prescribed source: presc[(step - presc0) * nJ + ...],
       either the whole arrays (pbox_on = 0) or a box of them (lo, ext) */
    double *presc;
    long presc_n, presc0;
    int pbox_on, pbox_lo[3], pbox_ext[3];
    /* adjoint state (reverse-time), same extents as the forward arrays */
    int adj_on;
    ofield Ea[3], Ha[3], Ja[3];
    ofield psiEa[3][3], psiHa[3][3];
    /* the material maps the coefficients were made from (C order) */
    double *wp_map, *gamma_map;
} osim;

static ofield fnew(int a, int b, int c)
{
    ofield f;
    f.n[0] = a;
    f.n[1] = b;
    f.n[2] = c;
    f.v = (double *)calloc((size_t)a * b * c + 1, sizeof(double));
    return f;
}

static void ffree(ofield *f)
{
    free(f->v);
    f->v = NULL;
}

static size_t fsize(const ofield *f) { return (size_t)f->n[0] * f->n[1] * f->n[2]; }

static double now_s(void)
{
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

/* Extents of component c: staggered (n cells) along c for E and across c for H. */
static void e_ext(const osim *s, int c, int e[3])
{
    for (int a = 0; a < 3; ++a) e[a] = s->n[a] + (a == c ? 0 : 1);
}
static void h_ext(const osim *s, int c, int e[3])
{
    for (int a = 0; a < 3; ++a) e[a] = s->n[a] + (a == c ? 1 : 0);
}

/*
 * CPML grading (Roden & Gedney 2000; the absorbing layer that stands in for
 * the Berenger PML of Sec. III).  Depth rho into a layer of thickness
 * L = npml dx, sigma = sigma_max (rho/L)^m, kappa = 1 + (kappa_max-1)(rho/L)^m,
 * alpha = alpha_max (1 - rho/L); b = exp(-(sigma/kappa + alpha) dt/eps0),
 * c = sigma (b-1) / (sigma kappa + kappa^2 alpha).
 */
static void cpml_coeff(const osim *s, int a, double pos, const double *pml, double *b,
                       double *c, double *kap, unsigned char *in)
{
    const double L = (double)s->npml;
    double rho = 0.0;
    if (pos < L) rho = L - pos;
    if (pos > (double)s->n[a] - L) rho = pos - ((double)s->n[a] - L);
    if (s->bc[a] != OR_CPML || s->npml <= 0 || rho <= 0.0) {
        *b = 1.0;
        *c = 0.0;
        *kap = 1.0;
        *in = 0;
        return;
    }
    const double m = pml[0];
    const double smax = pml[1] * 0.8 * (m + 1.0) / (OR_ETA0 * s->dx);
    const double r = rho / L;
    const double sig = smax * pow(r, m);
    const double kap_ = 1.0 + (pml[2] - 1.0) * pow(r, m);
    const double alp = pml[3] * (1.0 - r);
    *b = exp(-(sig / kap_ + alp) * s->dt / OR_EPS0);
    *c = (sig > 0.0) ? sig * (*b - 1.0) / (sig * kap_ + kap_ * kap_ * alp) : 0.0;
    *kap = kap_;
    *in = 1;
}

/*
 * Test-only: make axis a a uniform stretched coordinate with the given
 * recursion coefficients at every E-type and H-type position (so a periodic
 * axis stays translation invariant), allocating the memories it needs.  The
 * step's arithmetic is untouched; only its coefficient tables change.
 */
void osim_test_uniform_cpml(osim *s, int a, double b, double c, double kappa)
{
    for (int i = 0; i <= s->n[a]; ++i) {
        s->bE[a][i] = b;
        s->cE[a][i] = c;
        s->kE[a][i] = kappa;
        s->lE[a][i] = 1;
    }
    for (int i = 0; i < s->n[a]; ++i) {
        s->bH[a][i] = b;
        s->cH[a][i] = c;
        s->kH[a][i] = kappa;
        s->lH[a][i] = 1;
    }
    int e[3];
    for (int comp = 0; comp < 3; ++comp) {
        if (comp == a) continue;
        e_ext(s, comp, e);
        if (!s->psiE[comp][a].v) s->psiE[comp][a] = fnew(e[0], e[1], e[2]);
        h_ext(s, comp, e);
        if (!s->psiH[comp][a].v) s->psiH[comp][a] = fnew(e[0], e[1], e[2]);
    }
}

/* Test-only: copy out the coefficient tables of axis a (h = 0: E-type at
 * nodes 0..n, n+1 entries; h = 1: H-type at i+1/2, n entries). */
void osim_cpml_profile(const osim *s, int a, int h, double *b, double *c, double *kappa)
{
    const int len = h ? s->n[a] : s->n[a] + 1;
    for (int i = 0; i < len; ++i) {
        b[i] = h ? s->bH[a][i] : s->bE[a][i];
        c[i] = h ? s->cH[a][i] : s->cE[a][i];
        kappa[i] = h ? s->kH[a][i] : s->kE[a][i];
    }
}

/* Drude coefficients of Eq. 6 (c.f. the printed fractions). */
static void drude_coeff(double wp, double g, double dt, double *ca, double *cb)
{
    *ca = (2.0 - g * dt) / (2.0 + g * dt);
    *cb = 2.0 * dt * OR_EPS0 * wp * wp / (2.0 + g * dt);
}

/* Map (nx,ny,nz), C order (k fastest). */
static size_t cidx(const osim *s, int i, int j, int k)
{
    return ((size_t)i * s->n[1] + j) * s->n[2] + k;
}

static int clampi(int v, int hi) { return v < hi ? v : hi - 1; }

osim *osim_create(int nx, int ny, int nz, const int *bc, int npml, const double *pml,
                  double dx, double dt, const double *wp_map, const double *gamma_map)
{
    osim *s = (osim *)calloc(1, sizeof(osim));
    s->n[0] = nx;
    s->n[1] = ny;
    s->n[2] = nz;
    for (int a = 0; a < 3; ++a) s->bc[a] = bc[a];
    s->npml = npml;
    s->dx = dx;
    s->dt = dt;
    int e[3];
    for (int c = 0; c < 3; ++c) {
        e_ext(s, c, e);
        s->E[c] = fnew(e[0], e[1], e[2]);
        s->J[c] = fnew(e[0], e[1], e[2]);
        s->P[c] = fnew(e[0], e[1], e[2]);
        s->Jb[c] = fnew(e[0], e[1], e[2]);
        s->ca[c] = fnew(e[0], e[1], e[2]);
        s->cb[c] = fnew(e[0], e[1], e[2]);
        for (int a = 0; a < 3; ++a) s->psiE[c][a] = (a != c && bc[a] == OR_CPML) ? fnew(e[0], e[1], e[2]) : (ofield){{0, 0, 0}, NULL};
        h_ext(s, c, e);
        s->H[c] = fnew(e[0], e[1], e[2]);
        s->Hprev[c] = fnew(e[0], e[1], e[2]);
        for (int a = 0; a < 3; ++a) s->psiH[c][a] = (a != c && bc[a] == OR_CPML) ? fnew(e[0], e[1], e[2]) : (ofield){{0, 0, 0}, NULL};
    }
    /*
     * Edge material: cell (i,j,k) owns Ex(i+1/2,j,k), Ey(i,j+1/2,k),
     * Ez(i,j,k+1/2); edges on the upper walls take the last cell.  wp = 0
     * gives ca = 1, cb = 0 and J stays 0 in vacuum (Sec. II, after Eq. 8).
     */
    for (int c = 0; c < 3; ++c) {
        e_ext(s, c, e);
        for (int i = 0; i < e[0]; ++i)
            for (int j = 0; j < e[1]; ++j)
                for (int k = 0; k < e[2]; ++k) {
                    size_t m = cidx(s, clampi(i, nx), clampi(j, ny), clampi(k, nz));
                    drude_coeff(wp_map[m], gamma_map[m], dt, &AT(s->ca[c], i, j, k),
                                &AT(s->cb[c], i, j, k));
                }
    }
    s->wp_map = malloc(sizeof(double) * (size_t)nx * ny * nz);
    s->gamma_map = malloc(sizeof(double) * (size_t)nx * ny * nz);
    memcpy(s->wp_map, wp_map, sizeof(double) * (size_t)nx * ny * nz);
    memcpy(s->gamma_map, gamma_map, sizeof(double) * (size_t)nx * ny * nz);
    for (int a = 0; a < 3; ++a) {
        int n = s->n[a];
        s->bE[a] = calloc(n + 1, sizeof(double));
        s->cE[a] = calloc(n + 1, sizeof(double));
        s->kE[a] = calloc(n + 1, sizeof(double));
        s->lE[a] = calloc(n + 1, 1);
        s->bH[a] = calloc(n, sizeof(double));
        s->cH[a] = calloc(n, sizeof(double));
        s->kH[a] = calloc(n, sizeof(double));
        s->lH[a] = calloc(n, 1);
        for (int i = 0; i <= n; ++i)
            cpml_coeff(s, a, (double)i, pml, &s->bE[a][i], &s->cE[a][i], &s->kE[a][i], &s->lE[a][i]);
        for (int i = 0; i < n; ++i)
            cpml_coeff(s, a, i + 0.5, pml, &s->bH[a][i], &s->cH[a][i], &s->kH[a][i], &s->lH[a][i]);
    }
    return s;
}

void osim_destroy(osim *s)
{
    if (!s) return;
    for (int c = 0; c < 3; ++c) {
        ffree(&s->E[c]);
        ffree(&s->H[c]);
        ffree(&s->Hprev[c]);
        ffree(&s->J[c]);
        ffree(&s->P[c]);
        ffree(&s->Jb[c]);
        ffree(&s->ca[c]);
        ffree(&s->cb[c]);
        for (int a = 0; a < 3; ++a) {
            free(s->psiE[c][a].v);
            free(s->psiH[c][a].v);
        }
    }
    for (int a = 0; a < 3; ++a) {
        free(s->bE[a]);
        free(s->cE[a]);
        free(s->kE[a]);
        free(s->lE[a]);
        free(s->bH[a]);
        free(s->cH[a]);
        free(s->kH[a]);
        free(s->lH[a]);
    }
    free(s->x);
    free(s->y);
    free(s->z);
    free(s->ux);
    free(s->uy);
    free(s->uz);
    free(s->alive);
    free(s->pijk);
    free(s->omega);
    free(s->fre);
    free(s->fim);
    free(s->presc);
    free(s->wp_map);
    free(s->gamma_map);
    if (s->adj_on)
        for (int c = 0; c < 3; ++c) {
            ffree(&s->Ea[c]);
            ffree(&s->Ha[c]);
            ffree(&s->Ja[c]);
            for (int a = 0; a < 3; ++a) {
                free(s->psiEa[c][a].v);
                free(s->psiHa[c][a].v);
            }
        }
    free(s);
}

/* Raw state access: which 0=E 1=H 2=J_pol 3=P 4=J_b 5=H^{n-1/2} copy. */
double *osim_field_ptr(osim *s, int which, int comp, int *ext)
{
    ofield *f = NULL;
    switch (which) {
    case 0: f = &s->E[comp]; break;
    case 1: f = &s->H[comp]; break;
    case 2: f = &s->J[comp]; break;
    case 3: f = &s->P[comp]; break;
    case 4: f = &s->Jb[comp]; break;
    case 5: f = &s->Hprev[comp]; break;
    default: return NULL;
    }
    for (int a = 0; a < 3; ++a) ext[a] = f->n[a];
    return f->v;
}

/* Index of node/half-position `i` along axis a, folded for periodic axes. */
static int wrap(const osim *s, int a, int i)
{
    int n = s->n[a];
    return ((i % n) + n) % n;
}

/*
 * A tangential E edge on a PEC wall (also behind a CPML) is never updated;
 * on a periodic axis node n is the copy of node 0.
 */
static int e_node_updated(const osim *s, int a, int i)
{
    if (s->bc[a] == OR_PERIODIC) return i < s->n[a];
    return i > 0 && i < s->n[a];
}

/* ---- step 1: H in vacuum form, with CPML stretching in layer cells ---- */
static void update_H(osim *s)
{
    const double ch = s->dt / (OR_MU0 * s->dx);
    ofield Ex = s->E[0], Ey = s->E[1], Ez = s->E[2];
    for (int c = 0; c < 3; ++c) memcpy(s->Hprev[c].v, s->H[c].v, fsize(&s->H[c]) * sizeof(double));

    /* Hx(i, j+1/2, k+1/2) -= (dt/mu0) (dEz/dy - dEy/dz) */
    ofield Hx = s->H[0];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < Hx.n[0]; ++i)
        for (int j = 0; j < Hx.n[1]; ++j)
            for (int k = 0; k < Hx.n[2]; ++k) {
                double dy = AT(Ez, i, j + 1, k) - AT(Ez, i, j, k);
                double dz = AT(Ey, i, j, k + 1) - AT(Ey, i, j, k);
                if (s->lH[1][j]) {
                    double *p = &AT(s->psiH[0][1], i, j, k);
                    *p = s->bH[1][j] * *p + s->cH[1][j] * dy;
                    dy = dy / s->kH[1][j] + *p;
                }
                if (s->lH[2][k]) {
                    double *p = &AT(s->psiH[0][2], i, j, k);
                    *p = s->bH[2][k] * *p + s->cH[2][k] * dz;
                    dz = dz / s->kH[2][k] + *p;
                }
                AT(Hx, i, j, k) -= ch * (dy - dz);
            }
    /* Hy(i+1/2, j, k+1/2) -= (dt/mu0) (dEx/dz - dEz/dx) */
    ofield Hy = s->H[1];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < Hy.n[0]; ++i)
        for (int j = 0; j < Hy.n[1]; ++j)
            for (int k = 0; k < Hy.n[2]; ++k) {
                double dz = AT(Ex, i, j, k + 1) - AT(Ex, i, j, k);
                double dx = AT(Ez, i + 1, j, k) - AT(Ez, i, j, k);
                if (s->lH[2][k]) {
                    double *p = &AT(s->psiH[1][2], i, j, k);
                    *p = s->bH[2][k] * *p + s->cH[2][k] * dz;
                    dz = dz / s->kH[2][k] + *p;
                }
                if (s->lH[0][i]) {
                    double *p = &AT(s->psiH[1][0], i, j, k);
                    *p = s->bH[0][i] * *p + s->cH[0][i] * dx;
                    dx = dx / s->kH[0][i] + *p;
                }
                AT(Hy, i, j, k) -= ch * (dz - dx);
            }
    /* Hz(i+1/2, j+1/2, k) -= (dt/mu0) (dEy/dx - dEx/dy) */
    ofield Hz = s->H[2];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < Hz.n[0]; ++i)
        for (int j = 0; j < Hz.n[1]; ++j)
            for (int k = 0; k < Hz.n[2]; ++k) {
                double dx = AT(Ey, i + 1, j, k) - AT(Ey, i, j, k);
                double dy = AT(Ex, i, j + 1, k) - AT(Ex, i, j, k);
                if (s->lH[0][i]) {
                    double *p = &AT(s->psiH[2][0], i, j, k);
                    *p = s->bH[0][i] * *p + s->cH[0][i] * dx;
                    dx = dx / s->kH[0][i] + *p;
                }
                if (s->lH[1][j]) {
                    double *p = &AT(s->psiH[2][1], i, j, k);
                    *p = s->bH[1][j] * *p + s->cH[1][j] * dy;
                    dy = dy / s->kH[1][j] + *p;
                }
                AT(Hz, i, j, k) -= ch * (dx - dy);
            }
}

/* ---- steps 3+4: Eq. 6 then Eq. 8 on every updated E edge ---- */
static void update_E(osim *s)
{
    const double ce = s->dt / (OR_EPS0 * s->dx);
    const double cj = s->dt / OR_EPS0;
    const double dt = s->dt;
    ofield Hx = s->H[0], Hy = s->H[1], Hz = s->H[2];

    /* Ex(i+1/2, j, k) += (dt/eps0) (dHz/dy - dHy/dz - J - Jb) */
    ofield Ex = s->E[0];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < Ex.n[0]; ++i)
        for (int j = 0; j < Ex.n[1]; ++j)
            for (int k = 0; k < Ex.n[2]; ++k) {
                if (!e_node_updated(s, 1, j) || !e_node_updated(s, 2, k)) continue;
                int jm = wrap(s, 1, j - 1), km = wrap(s, 2, k - 1);
                double dy = AT(Hz, i, j, k) - AT(Hz, i, jm, k);
                double dz = AT(Hy, i, j, k) - AT(Hy, i, j, km);
                if (s->lE[1][j]) {
                    double *p = &AT(s->psiE[0][1], i, j, k);
                    *p = s->bE[1][j] * *p + s->cE[1][j] * dy;
                    dy = dy / s->kE[1][j] + *p;
                }
                if (s->lE[2][k]) {
                    double *p = &AT(s->psiE[0][2], i, j, k);
                    *p = s->bE[2][k] * *p + s->cE[2][k] * dz;
                    dz = dz / s->kE[2][k] + *p;
                }
                double jn = AT(s->ca[0], i, j, k) * AT(s->J[0], i, j, k) + AT(s->cb[0], i, j, k) * AT(Ex, i, j, k);
                AT(s->J[0], i, j, k) = jn;
                AT(s->P[0], i, j, k) += dt * jn;
                AT(Ex, i, j, k) += ce * (dy - dz) - cj * (jn + AT(s->Jb[0], i, j, k));
            }
    /* Ey(i, j+1/2, k) += (dt/eps0) (dHx/dz - dHz/dx - J - Jb) */
    ofield Ey = s->E[1];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < Ey.n[0]; ++i)
        for (int j = 0; j < Ey.n[1]; ++j)
            for (int k = 0; k < Ey.n[2]; ++k) {
                if (!e_node_updated(s, 0, i) || !e_node_updated(s, 2, k)) continue;
                int im = wrap(s, 0, i - 1), km = wrap(s, 2, k - 1);
                double dz = AT(Hx, i, j, k) - AT(Hx, i, j, km);
                double dx = AT(Hz, i, j, k) - AT(Hz, im, j, k);
                if (s->lE[2][k]) {
                    double *p = &AT(s->psiE[1][2], i, j, k);
                    *p = s->bE[2][k] * *p + s->cE[2][k] * dz;
                    dz = dz / s->kE[2][k] + *p;
                }
                if (s->lE[0][i]) {
                    double *p = &AT(s->psiE[1][0], i, j, k);
                    *p = s->bE[0][i] * *p + s->cE[0][i] * dx;
                    dx = dx / s->kE[0][i] + *p;
                }
                double jn = AT(s->ca[1], i, j, k) * AT(s->J[1], i, j, k) + AT(s->cb[1], i, j, k) * AT(Ey, i, j, k);
                AT(s->J[1], i, j, k) = jn;
                AT(s->P[1], i, j, k) += dt * jn;
                AT(Ey, i, j, k) += ce * (dz - dx) - cj * (jn + AT(s->Jb[1], i, j, k));
            }
    /* Ez(i, j, k+1/2) += (dt/eps0) (dHy/dx - dHx/dy - J - Jb) */
    ofield Ez = s->E[2];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < Ez.n[0]; ++i)
        for (int j = 0; j < Ez.n[1]; ++j)
            for (int k = 0; k < Ez.n[2]; ++k) {
                if (!e_node_updated(s, 0, i) || !e_node_updated(s, 1, j)) continue;
                int im = wrap(s, 0, i - 1), jm = wrap(s, 1, j - 1);
                double dx = AT(Hy, i, j, k) - AT(Hy, im, j, k);
                double dy = AT(Hx, i, j, k) - AT(Hx, i, jm, k);
                if (s->lE[0][i]) {
                    double *p = &AT(s->psiE[2][0], i, j, k);
                    *p = s->bE[0][i] * *p + s->cE[0][i] * dx;
                    dx = dx / s->kE[0][i] + *p;
                }
                if (s->lE[1][j]) {
                    double *p = &AT(s->psiE[2][1], i, j, k);
                    *p = s->bE[1][j] * *p + s->cE[1][j] * dy;
                    dy = dy / s->kE[1][j] + *p;
                }
                double jn = AT(s->ca[2], i, j, k) * AT(s->J[2], i, j, k) + AT(s->cb[2], i, j, k) * AT(Ez, i, j, k);
                AT(s->J[2], i, j, k) = jn;
                AT(s->P[2], i, j, k) += dt * jn;
                AT(Ez, i, j, k) += ce * (dx - dy) - cj * (jn + AT(s->Jb[2], i, j, k));
            }
    /* Periodic copies: node n of a non-staggered periodic axis mirrors node 0. */
    for (int c = 0; c < 3; ++c) {
        ofield f = s->E[c];
        for (int a = 0; a < 3; ++a) {
            if (a == c || s->bc[a] != OR_PERIODIC) continue;
            int n = s->n[a];
            for (int i = 0; i < f.n[0]; ++i)
                for (int j = 0; j < f.n[1]; ++j)
                    for (int k = 0; k < f.n[2]; ++k) {
                        int id[3] = {i, j, k};
                        if (id[a] != n) continue;
                        id[a] = 0;
                        AT(f, i, j, k) = AT(f, id[0], id[1], id[2]);
                    }
        }
        memset(s->Jb[c].v, 0, fsize(&s->Jb[c]) * sizeof(double));
    }
}

/* ---- particles ---- */

/* Value of a stored component at integer lattice index, 0 outside the box. */
static double fetch(const osim *s, const ofield *f, int i, int j, int k)
{
    int id[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        if (s->bc[a] == OR_PERIODIC) {
            id[a] = wrap(s, a, id[a]);
        } else if (id[a] < 0 || id[a] >= f->n[a]) {
            return 0.0;
        }
    }
    return AT(*f, id[0], id[1], id[2]);
}

/*
 * Trilinear (cloud-in-cell) interpolation of one component on its own
 * staggered lattice; off[a] = 1/2 on the axes where it sits at half cells.
 * X is in cell units.
 */
static double interp(const osim *s, const ofield *f, const double off[3], const double X[3])
{
    int i0[3];
    double fr[3];
    for (int a = 0; a < 3; ++a) {
        double t = X[a] - off[a];
        i0[a] = (int)floor(t);
        fr[a] = t - i0[a];
    }
    double v = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
                double wgt = (a ? fr[0] : 1.0 - fr[0]) * (b ? fr[1] : 1.0 - fr[1]) * (c ? fr[2] : 1.0 - fr[2]);
                v += wgt * fetch(s, f, i0[0] + a, i0[1] + b, i0[2] + c);
            }
    return v;
}

/* E^n and B^n = mu0 (H^{n-1/2} + H^{n+1/2})/2 at a point given in metres. */
void osim_gather(const osim *s, const double *pos, double *E, double *B)
{
    double X[3] = {pos[0] / s->dx, pos[1] / s->dx, pos[2] / s->dx};
    for (int c = 0; c < 3; ++c) {
        double oe[3] = {0, 0, 0}, oh[3] = {0.5, 0.5, 0.5};
        oe[c] = 0.5;
        oh[c] = 0.0;
        E[c] = interp(s, &s->E[c], oe, X);
        B[c] = OR_MU0 * 0.5 * (interp(s, &s->Hprev[c], oh, X) + interp(s, &s->H[c], oh, X));
    }
}

/*
 * Relativistic Boris rotation (Boris 1970; Birdsall & Langdon Sec. 15-4).
 * u = gamma v in m/s, advanced from n-1/2 to n+1/2 under E, B at time n.
 */
void oracle_boris(double q, double m, double dt, const double *E, const double *B, double *u)
{
    const double h = q * dt / (2.0 * m);
    double um[3], t[3], sv[3], up[3], uq[3];
    for (int a = 0; a < 3; ++a) um[a] = u[a] + h * E[a];
    double g = sqrt(1.0 + (um[0] * um[0] + um[1] * um[1] + um[2] * um[2]) / (OR_C * OR_C));
    for (int a = 0; a < 3; ++a) t[a] = h * B[a] / g;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int a = 0; a < 3; ++a) sv[a] = 2.0 * t[a] / (1.0 + t2);
    up[0] = um[0] + (um[1] * t[2] - um[2] * t[1]);
    up[1] = um[1] + (um[2] * t[0] - um[0] * t[2]);
    up[2] = um[2] + (um[0] * t[1] - um[1] * t[0]);
    uq[0] = um[0] + (up[1] * sv[2] - up[2] * sv[1]);
    uq[1] = um[1] + (up[2] * sv[0] - up[0] * sv[2]);
    uq[2] = um[2] + (up[0] * sv[1] - up[1] * sv[0]);
    for (int a = 0; a < 3; ++a) u[a] = uq[a] + h * E[a];
}

static double shape1(double t)
{
    double a = fabs(t);
    return a < 1.0 ? 1.0 - a : 0.0;
}

static void add_at(osim *s, ofield *f, int i, int j, int k, double v)
{
    int id[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        if (s->bc[a] == OR_PERIODIC) id[a] = wrap(s, a, id[a]);
        else if (id[a] < 0 || id[a] >= f->n[a]) return;
    }
    AT(*f, id[0], id[1], id[2]) += v;
}

/*
 * A copy of the three bunch-current arrays over a box of lattice indices
 * lo .. lo + ext - 1 per axis (unwrapped: indices may lie one node outside
 * the grid), components back to back, x slowest.  Deposits land here first;
 * jbox_flush adds the box to J_b, wrapping periodic axes and dropping what
 * lies outside the grid.
 */
typedef struct {
    double *v;
    int lo[3], ext[3];
} jbox;

static void jbox_add(jbox *b, int c, int i, int j, int k, double v)
{
    const size_t q = (((size_t)c * b->ext[0] + (size_t)(i - b->lo[0])) * b->ext[1] + (size_t)(j - b->lo[1])) *
                         b->ext[2] +
                     (size_t)(k - b->lo[2]);
    b->v[q] += v;
}

static void jbox_flush(osim *s, const jbox *b)
{
    size_t q = 0;
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < b->ext[0]; ++i)
            for (int j = 0; j < b->ext[1]; ++j)
                for (int k = 0; k < b->ext[2]; ++k, ++q)
                    if (b->v[q] != 0.0) add_at(s, &s->Jb[c], b->lo[0] + i, b->lo[1] + j, b->lo[2] + k, b->v[q]);
}

/*
 * Charge-conserving deposit of one macro-particle moving X0 -> X1 (cell
 * units), Esirkepov, Comput. Phys. Commun. 135 (2001) 144, first-order
 * shape S(t) = max(0, 1-|t|) at the nodes.  Over a 4-node window per axis
 * starting one node below the start cell:
 *   Wx = dSx (S0y S0z + dSy S0z/2 + S0y dSz/2 + dSy dSz/3)   (and cyclic),
 *   Jx(i+1/2) = -(q w / (dt dx^2)) sum_{i' <= i} Wx(i')      (and cyclic).
 * The window must lie inside the box.
 */
static void deposit(osim *s, jbox *box, const double *X0, const double *X1, double qw)
{
    int base[3];
    double S0[3][4], S1[3][4], dS[3][4];
    for (int a = 0; a < 3; ++a) {
        base[a] = (int)floor(X0[a]) - 1;
        for (int m = 0; m < 4; ++m) {
            S0[a][m] = shape1(X0[a] - (base[a] + m));
            S1[a][m] = shape1(X1[a] - (base[a] + m));
            dS[a][m] = S1[a][m] - S0[a][m];
        }
    }
    const double f = -qw / (s->dt * s->dx * s->dx);
    for (int b = 0; b < 4; ++b)
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
            for (int m = 0; m < 3; ++m) {
                acc += dS[0][m] * (S0[1][b] * S0[2][c] + 0.5 * dS[1][b] * S0[2][c] +
                                   0.5 * S0[1][b] * dS[2][c] + dS[1][b] * dS[2][c] / 3.0);
                jbox_add(box, 0, base[0] + m, base[1] + b, base[2] + c, f * acc);
            }
        }
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) {
            double acc = 0.0;
            for (int m = 0; m < 3; ++m) {
                acc += dS[1][m] * (S0[0][a] * S0[2][c] + 0.5 * dS[0][a] * S0[2][c] +
                                   0.5 * S0[0][a] * dS[2][c] + dS[0][a] * dS[2][c] / 3.0);
                jbox_add(box, 1, base[0] + a, base[1] + m, base[2] + c, f * acc);
            }
        }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            double acc = 0.0;
            for (int m = 0; m < 3; ++m) {
                acc += dS[2][m] * (S0[0][a] * S0[1][b] + 0.5 * dS[0][a] * S0[1][b] +
                                   0.5 * S0[0][a] * dS[1][b] + dS[0][a] * dS[1][b] / 3.0);
                jbox_add(box, 2, base[0] + a, base[1] + b, base[2] + m, f * acc);
            }
        }
}

/* Deposit one move given in metres into J_b with the configured q w. */
void osim_deposit_move(osim *s, const double *p0, const double *p1)
{
    double X0[3], X1[3];
    jbox box;
    for (int a = 0; a < 3; ++a) {
        X0[a] = p0[a] / s->dx;
        X1[a] = p1[a] / s->dx;
        box.lo[a] = (int)floor(X0[a]) - 1;
        box.ext[a] = 4;
    }
    box.v = calloc(3 * 64, sizeof(double));
    deposit(s, &box, X0, X1, s->q * s->w);
    jbox_flush(s, &box);
    free(box.v);
}

/* Gather, Boris, move and deposit of live particle p; 1 if its move was
 * deposited, 0 if it left the box. */
static int push_one(osim *s, jbox *box, long p)
{
    const double dx = s->dx;
    double pos[3] = {s->x[p], s->y[p], s->z[p]};
    double E[3], B[3], u[3] = {s->ux[p], s->uy[p], s->uz[p]};
    osim_gather(s, pos, E, B);
    oracle_boris(s->q, s->m, s->dt, E, B, u);
    double g = sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / (OR_C * OR_C));
    double X0[3], X1[3];
    int out = 0;
    for (int a = 0; a < 3; ++a) {
        X0[a] = pos[a] / dx;
        X1[a] = (pos[a] + s->dt * u[a] / g) / dx;
        if (s->bc[a] != OR_PERIODIC && (X1[a] < 0.0 || X1[a] >= (double)s->n[a])) out = 1;
    }
    s->ux[p] = u[0];
    s->uy[p] = u[1];
    s->uz[p] = u[2];
    if (out) {
        s->alive[p] = 0;
        return 0;
    }
    deposit(s, box, X0, X1, s->q * s->w);
    for (int a = 0; a < 3; ++a) {
        if (s->bc[a] == OR_PERIODIC) {
            double L = (double)s->n[a];
            X1[a] = fmod(X1[a], L);
            if (X1[a] < 0.0) X1[a] += L;
        }
    }
    s->x[p] = X1[0] * dx;
    s->y[p] = X1[1] * dx;
    s->z[p] = X1[2] * dx;
    return 1;
}

/* Particles per chunk of the push; below this count one chunk does all. */
#define OR_CHUNK_MIN 4096
#define OR_NCHUNK 16

/*
 * Step 2: gather, push, move, deposit.  A particle whose new position leaves
 * [0, n dx) on a non-periodic axis is deactivated and its last move is not
 * deposited; on a periodic axis it is folded back after the deposit.
 *
 * The particles are split by index into a fixed number of chunks (one below
 * OR_CHUNK_MIN particles), which may run on different threads.  Each chunk
 * deposits into its own copy of J_b over the box of every deposit window of
 * this step, and the copies are added to J_b in chunk order, so the result
 * does not depend on the number of threads.
 */
static void push_particles(osim *s)
{
    jbox all;
    long nlive = 0;
    for (int a = 0; a < 3; ++a) {
        all.lo[a] = s->n[a];
        all.ext[a] = 0;
    }
    int hi[3] = {-1, -1, -1};
    for (long p = 0; p < s->np; ++p) {
        if (!s->alive[p]) continue;
        const double pos[3] = {s->x[p], s->y[p], s->z[p]};
        for (int a = 0; a < 3; ++a) {
            const int f = (int)floor(pos[a] / s->dx);
            if (f - 1 < all.lo[a]) all.lo[a] = f - 1;
            if (f + 2 > hi[a]) hi[a] = f + 2;
        }
        ++nlive;
    }
    if (nlive == 0) return;
    size_t cells = 1;
    for (int a = 0; a < 3; ++a) {
        all.ext[a] = hi[a] - all.lo[a] + 1;
        cells *= (size_t)all.ext[a];
    }
    const int nchunk = s->np >= OR_CHUNK_MIN ? OR_NCHUNK : 1;
    double *buf = calloc((size_t)nchunk * 3 * cells, sizeof(double));
    long pushed[OR_NCHUNK] = {0};
#pragma omp parallel for schedule(dynamic, 1)
    for (int ch = 0; ch < nchunk; ++ch) {
        jbox box = all;
        box.v = buf + (size_t)ch * 3 * cells;
        const long p0 = s->np * ch / nchunk, p1 = s->np * (ch + 1) / nchunk;
        for (long p = p0; p < p1; ++p)
            if (s->alive[p]) pushed[ch] += push_one(s, &box, p);
    }
    for (int ch = 0; ch < nchunk; ++ch) {
        jbox box = all;
        box.v = buf + (size_t)ch * 3 * cells;
        jbox_flush(s, &box);
        s->pushes += pushed[ch];
    }
    free(buf);
}


void osim_set_particles(osim *s, long n, const double *x, const double *y, const double *z,
                        const double *ux, const double *uy, const double *uz, double q, double m,
                        double w)
{
    free(s->x);
    free(s->y);
    free(s->z);
    free(s->ux);
    free(s->uy);
    free(s->uz);
    free(s->alive);
    s->np = n;
    size_t b = (size_t)(n > 0 ? n : 1) * sizeof(double);
    s->x = malloc(b);
    s->y = malloc(b);
    s->z = malloc(b);
    s->ux = malloc(b);
    s->uy = malloc(b);
    s->uz = malloc(b);
    s->alive = malloc(n > 0 ? n : 1);
    for (long p = 0; p < n; ++p) {
        s->x[p] = x[p];
        s->y[p] = y[p];
        s->z[p] = z[p];
        s->ux[p] = ux[p];
        s->uy[p] = uy[p];
        s->uz[p] = uz[p];
        s->alive[p] = 1;
    }
    s->q = q;
    s->m = m;
    s->w = w;
}

/* which: 0..5 = x y z ux uy uz (copy out); alive flags as 0/1 doubles for 6. */
void osim_get_particles(const osim *s, int which, double *out)
{
    const double *src[6] = {s->x, s->y, s->z, s->ux, s->uy, s->uz};
    for (long p = 0; p < s->np; ++p) out[p] = which < 6 ? src[which][p] : (double)s->alive[p];
}

/*
 * Probes sample the nearest Ez node (i, j, k+1/2): i, j round half up,
 * k = floor(z/dx) (ties toward +z).
 */
void osim_set_probes(osim *s, int nprobe, const double *xyz, int nfreq, const double *omega)
{
    free(s->pijk);
    free(s->omega);
    free(s->fre);
    free(s->fim);
    s->nprobe = nprobe;
    s->nfreq = nfreq;
    s->pijk = calloc(3 * (size_t)(nprobe > 0 ? nprobe : 1), sizeof(int));
    s->omega = calloc((size_t)(nfreq > 0 ? nfreq : 1), sizeof(double));
    s->fre = calloc((size_t)(nprobe * nfreq > 0 ? nprobe * nfreq : 1), sizeof(double));
    s->fim = calloc((size_t)(nprobe * nfreq > 0 ? nprobe * nfreq : 1), sizeof(double));
    for (int p = 0; p < nprobe; ++p) {
        s->pijk[3 * p + 0] = (int)floor(xyz[3 * p + 0] / s->dx + 0.5);
        s->pijk[3 * p + 1] = (int)floor(xyz[3 * p + 1] / s->dx + 0.5);
        s->pijk[3 * p + 2] = (int)floor(xyz[3 * p + 2] / s->dx);
    }
    for (int f = 0; f < nfreq; ++f) s->omega[f] = omega[f];
}

static void sample_probes(osim *s)
{
    const double t = (double)s->step * s->dt; /* time of E^{n+1}, step already advanced */
    for (int p = 0; p < s->nprobe; ++p) {
        double ez = AT(s->E[2], s->pijk[3 * p], s->pijk[3 * p + 1], s->pijk[3 * p + 2]);
        for (int f = 0; f < s->nfreq; ++f) {
            double th = s->omega[f] * t;
            s->fre[p * s->nfreq + f] += s->dt * ez * cos(th);
            s->fim[p * s->nfreq + f] -= s->dt * ez * sin(th);
        }
    }
}

void osim_probe(const osim *s, double *re, double *im)
{
    for (int i = 0; i < s->nprobe * s->nfreq; ++i) {
        re[i] = s->fre[i];
        im[i] = s->fim[i];
    }
}

/* Probe Ez values of the current E (for time series). */
void osim_probe_values(const osim *s, double *out)
{
    for (int p = 0; p < s->nprobe; ++p)
        out[p] = AT(s->E[2], s->pijk[3 * p], s->pijk[3 * p + 1], s->pijk[3 * p + 2]);
}

/* Number of doubles in one J_b snapshot (the three components back to back). */
long osim_jb_size(const osim *s)
{
    return (long)(fsize(&s->Jb[0]) + fsize(&s->Jb[1]) + fsize(&s->Jb[2]));
}

static void jb_save(const osim *s, double *out)
{
    size_t o = 0;
    for (int c = 0; c < 3; ++c) {
        memcpy(out + o, s->Jb[c].v, fsize(&s->Jb[c]) * sizeof(double));
        o += fsize(&s->Jb[c]);
    }
}

static void jb_load(osim *s, const double *in)
{
    size_t o = 0;
    for (int c = 0; c < 3; ++c) {
        memcpy(s->Jb[c].v, in + o, fsize(&s->Jb[c]) * sizeof(double));
        o += fsize(&s->Jb[c]);
    }
}

/*
 * From now on use the given bunch current J_b^{n+1/2} for the next n steps
 * instead of pushing particles (the source held fixed by the adjoint).
 */
void osim_prescribe_jb(osim *s, const double *hist, long n)
{
    s->pbox_on = 0;
    free(s->presc);
    s->presc = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * (size_t)osim_jb_size(s));
    memcpy(s->presc, hist, sizeof(double) * (size_t)n * (size_t)osim_jb_size(s));
    s->presc_n = n;
    s->presc0 = s->step;
}

/* Entries of one box record: the box [lo, lo + ext) of each J_b component. */
static size_t jbox_count(const int *ext) { return (size_t)3 * ext[0] * ext[1] * ext[2]; }

/* Copy the box of J_b to out (component, then x, y, z with z fastest), or
 * back; box entries beyond a component's own extents hold 0. */
static void jb_box_copy(osim *s, const int *lo, const int *ext, double *buf, int to_grid)
{
    size_t q = 0;
    for (int c = 0; c < 3; ++c)
        for (int i = 0; i < ext[0]; ++i)
            for (int j = 0; j < ext[1]; ++j)
                for (int k = 0; k < ext[2]; ++k, ++q) {
                    const int id[3] = {lo[0] + i, lo[1] + j, lo[2] + k};
                    if (id[0] >= s->Jb[c].n[0] || id[1] >= s->Jb[c].n[1] || id[2] >= s->Jb[c].n[2]) {
                        if (!to_grid) buf[q] = 0.0;
                        continue;
                    }
                    double *v = &AT(s->Jb[c], id[0], id[1], id[2]);
                    if (to_grid) *v = buf[q];
                    else buf[q] = *v;
                }
}

/* Step 2 of the step: particles, or the prescribed bunch current. */
static void source_step(osim *s)
{
    if (s->presc) {
        long r = s->step - s->presc0;
        if (r >= 0 && r < s->presc_n) {
            if (s->pbox_on)
                jb_box_copy(s, s->pbox_lo, s->pbox_ext, s->presc + (size_t)r * jbox_count(s->pbox_ext), 1);
            else
                jb_load(s, s->presc + (size_t)r * (size_t)osim_jb_size(s));
        }
    } else {
        push_particles(s);
    }
}

/*
 * Run n steps from the current state and record J_b^{n+1/2} of each step on
 * the box [lo, lo + ext) of lattice indices (0 <= lo, lo + ext <= n + 1 per
 * axis; clipped to each component's extents): out[n][3][ext0][ext1][ext2].  Returns the largest |J_b| met outside the
 * box during the run (0 when the box holds every deposit).
 */
double osim_run_record_jb_box(osim *s, long n, const int *lo, const int *ext, double *out)
{
    const size_t nb = jbox_count(ext);
    double outside = 0.0;
    for (long it = 0; it < n; ++it) {
        update_H(s);
        source_step(s);
        jb_box_copy(s, lo, ext, out + (size_t)it * nb, 0);
        for (int c = 0; c < 3; ++c) {
            const ofield *f = &s->Jb[c];
            for (int i = 0; i < f->n[0]; ++i)
                for (int j = 0; j < f->n[1]; ++j)
                    for (int k = 0; k < f->n[2]; ++k) {
                        const int in = i >= lo[0] && i < lo[0] + ext[0] && j >= lo[1] && j < lo[1] + ext[1] &&
                                       k >= lo[2] && k < lo[2] + ext[2];
                        const double v = fabs(AT(*f, i, j, k));
                        if (!in && v > outside) outside = v;
                    }
        }
        update_E(s);
        s->step++;
        sample_probes(s);
    }
    return outside;
}

/* Use the box records of osim_run_record_jb_box as the bunch current of the
 * next n steps (zero outside the box) instead of pushing particles. */
void osim_prescribe_jb_box(osim *s, const int *lo, const int *ext, const double *hist, long n)
{
    const size_t nb = jbox_count(ext);
    free(s->presc);
    s->presc = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * nb);
    memcpy(s->presc, hist, sizeof(double) * (size_t)n * nb);
    s->presc_n = n;
    s->presc0 = s->step;
    s->pbox_on = 1;
    for (int a = 0; a < 3; ++a) {
        s->pbox_lo[a] = lo[a];
        s->pbox_ext[a] = ext[a];
    }
}

void osim_step(osim *s, long nsteps)
{
    for (long it = 0; it < nsteps; ++it) {
        double t0 = now_s();
        update_H(s);
        double t1 = now_s();
        source_step(s);
        double t2 = now_s();
        update_E(s);
        s->step++;
        sample_probes(s);
        double t3 = now_s();
        s->t_field += (t1 - t0) + (t3 - t2);
        s->t_part += t2 - t1;
    }
}

long osim_get_step(const osim *s) { return s->step; }

/* out[0] field seconds, out[1] particle seconds, out[2] pushes, out[3] threads */
void osim_timing(const osim *s, double *out)
{
    out[0] = s->t_field;
    out[1] = s->t_part;
    out[2] = (double)s->pushes;
#ifdef _OPENMP
    out[3] = (double)omp_get_max_threads();
#else
    out[3] = 1.0;
#endif
}

/* ---- diagnostics ---- */

/* Node-centred CIC charge density rho on the (nx+1)(ny+1)(nz+1) nodes. */
void osim_rho(const osim *s, double *rho)
{
    const int n1 = s->n[1] + 1, n2 = s->n[2] + 1;
    memset(rho, 0, sizeof(double) * (size_t)(s->n[0] + 1) * n1 * n2);
    const double v = s->dx * s->dx * s->dx;
    for (long p = 0; p < s->np; ++p) {
        if (!s->alive[p]) continue;
        double X[3] = {s->x[p] / s->dx, s->y[p] / s->dx, s->z[p] / s->dx};
        int i0[3];
        double fr[3];
        for (int a = 0; a < 3; ++a) {
            i0[a] = (int)floor(X[a]);
            fr[a] = X[a] - i0[a];
        }
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) {
                    int id[3] = {i0[0] + a, i0[1] + b, i0[2] + c};
                    int skip = 0;
                    for (int d = 0; d < 3; ++d) {
                        if (s->bc[d] == OR_PERIODIC) id[d] = wrap(s, d, id[d]);
                        else if (id[d] < 0 || id[d] > s->n[d]) skip = 1;
                    }
                    if (skip) continue;
                    double wgt = (a ? fr[0] : 1 - fr[0]) * (b ? fr[1] : 1 - fr[1]) * (c ? fr[2] : 1 - fr[2]);
                    rho[((size_t)id[0] * n1 + id[1]) * n2 + id[2]] += s->q * s->w * wgt / v;
                }
    }
}

/*
 * Gauss-law residual G = eps0 div E + div P - rho at interior nodes
 * (1..n-1 on every axis; 0 elsewhere), with P^{n+1} = P^n + dt J^{n+1/2}
 * the polarization of Eq. 2 accumulated from the Drude current.
 */
void osim_gauss(const osim *s, double *G)
{
    const int n0 = s->n[0] + 1, n1 = s->n[1] + 1, n2 = s->n[2] + 1;
    double *rho = malloc(sizeof(double) * (size_t)n0 * n1 * n2);
    osim_rho(s, rho);
    memset(G, 0, sizeof(double) * (size_t)n0 * n1 * n2);
    for (int i = 1; i < s->n[0]; ++i)
        for (int j = 1; j < s->n[1]; ++j)
            for (int k = 1; k < s->n[2]; ++k) {
                double dE = (AT(s->E[0], i, j, k) - AT(s->E[0], i - 1, j, k)) +
                            (AT(s->E[1], i, j, k) - AT(s->E[1], i, j - 1, k)) +
                            (AT(s->E[2], i, j, k) - AT(s->E[2], i, j, k - 1));
                double dP = (AT(s->P[0], i, j, k) - AT(s->P[0], i - 1, j, k)) +
                            (AT(s->P[1], i, j, k) - AT(s->P[1], i, j - 1, k)) +
                            (AT(s->P[2], i, j, k) - AT(s->P[2], i, j, k - 1));
                size_t m = ((size_t)i * n1 + j) * n2 + k;
                G[m] = (OR_EPS0 * dE + dP) / s->dx - rho[m];
            }
    free(rho);
}

/*
 * Field energy (eps0 |E|^2 + mu0 |H|^2)/2 dx^3 summed over stored edges and
 * faces (periodic copies at node n excluded), and bunch moments over the
 * live particles: out = [energy, count, <x>,<y>,<z>, sx,sy,sz, <ux>,<uy>,<uz>].
 */
void osim_diag(const osim *s, double *out)
{
    double en = 0.0;
    for (int which = 0; which < 2; ++which)
        for (int c = 0; c < 3; ++c) {
            const ofield *f = which ? &s->H[c] : &s->E[c];
            const double coef = which ? OR_MU0 : OR_EPS0;
            for (int i = 0; i < f->n[0]; ++i)
                for (int j = 0; j < f->n[1]; ++j)
                    for (int k = 0; k < f->n[2]; ++k) {
                        int id[3] = {i, j, k};
                        int dup = 0;
                        for (int a = 0; a < 3; ++a)
                            if (s->bc[a] == OR_PERIODIC && id[a] == s->n[a]) dup = 1;
                        if (dup) continue;
                        double v = AT(*f, i, j, k);
                        en += 0.5 * coef * v * v;
                    }
        }
    out[0] = en * s->dx * s->dx * s->dx;
    double cnt = 0, mx[3] = {0, 0, 0}, m2[3] = {0, 0, 0}, mu[3] = {0, 0, 0};
    for (long p = 0; p < s->np; ++p) {
        if (!s->alive[p]) continue;
        double v[3] = {s->x[p], s->y[p], s->z[p]}, u[3] = {s->ux[p], s->uy[p], s->uz[p]};
        cnt += 1;
        for (int a = 0; a < 3; ++a) {
            mx[a] += v[a];
            m2[a] += v[a] * v[a];
            mu[a] += u[a];
        }
    }
    out[1] = cnt;
    for (int a = 0; a < 3; ++a) {
        double mean = cnt > 0 ? mx[a] / cnt : 0.0;
        double var = cnt > 0 ? m2[a] / cnt - mean * mean : 0.0;
        out[2 + a] = mean;
        out[5 + a] = var > 0 ? sqrt(var) : 0.0;
        out[8 + a] = cnt > 0 ? mu[a] / cnt : 0.0;
    }
}

/* Physical constants the oracle uses: c, mu0, eps0. */
void oracle_constants(double *out)
{
    out[0] = OR_C;
    out[1] = OR_MU0;
    out[2] = OR_EPS0;
}

/* ======================================================================
 * Adjoint (reverse-time) of the field + Drude + CPML step with the bunch
 * current held fixed, and the gradient of the probe spectral power
 *   L = sum_p |F_p(w0)|^2,   F_p = sum_{n=1..N} dt Ez_p^n exp(-i w0 n dt)
 * with respect to the per-cell plasma and collision frequencies (the maps
 * of Eq. 1).  The step is linear in (E, H, J, psi); its transpose is taken
 * operation by operation in reverse order.  For a forward update of the form
 *   psi' = b psi + c d,   t = d / kappa + psi',   X' = X + s t
 * the adjoint, given Xbar' and psibar' (from later steps), is
 *   tbar = s Xbar',  psibar_tot = psibar' + tbar,
 *   dbar = tbar / kappa + c psibar_tot,  psibar = b psibar_tot,
 * and dbar is scattered onto the two values whose difference is d.
 * ====================================================================== */

static void adj_alloc(osim *s)
{
    if (s->adj_on) return;
    for (int c = 0; c < 3; ++c) {
        s->Ea[c] = fnew(s->E[c].n[0], s->E[c].n[1], s->E[c].n[2]);
        s->Ja[c] = fnew(s->E[c].n[0], s->E[c].n[1], s->E[c].n[2]);
        s->Ha[c] = fnew(s->H[c].n[0], s->H[c].n[1], s->H[c].n[2]);
        for (int a = 0; a < 3; ++a) {
            s->psiEa[c][a] = s->psiE[c][a].v ? fnew(s->E[c].n[0], s->E[c].n[1], s->E[c].n[2]) : (ofield){{0, 0, 0}, NULL};
            s->psiHa[c][a] = s->psiH[c][a].v ? fnew(s->H[c].n[0], s->H[c].n[1], s->H[c].n[2]) : (ofield){{0, 0, 0}, NULL};
        }
    }
    s->adj_on = 1;
}

void osim_adj_zero(osim *s)
{
    adj_alloc(s);
    for (int c = 0; c < 3; ++c) {
        memset(s->Ea[c].v, 0, fsize(&s->Ea[c]) * sizeof(double));
        memset(s->Ja[c].v, 0, fsize(&s->Ja[c]) * sizeof(double));
        memset(s->Ha[c].v, 0, fsize(&s->Ha[c]) * sizeof(double));
        for (int a = 0; a < 3; ++a) {
            if (s->psiEa[c][a].v) memset(s->psiEa[c][a].v, 0, fsize(&s->psiEa[c][a]) * sizeof(double));
            if (s->psiHa[c][a].v) memset(s->psiHa[c][a].v, 0, fsize(&s->psiHa[c][a]) * sizeof(double));
        }
    }
}

/*
 * Raw access: which 0 = E-bar, 1 = H-bar, 2 = J-bar (comp c), 3 = psi_E,
 * 4 = psi_H, 5 = psi_E-bar, 6 = psi_H-bar (comp c, derivative axis a).
 * NULL when the array does not exist.
 */
double *osim_adj_ptr(osim *s, int which, int c, int a, int *ext)
{
    adj_alloc(s);
    ofield *f = NULL;
    switch (which) {
    case 0: f = &s->Ea[c]; break;
    case 1: f = &s->Ha[c]; break;
    case 2: f = &s->Ja[c]; break;
    case 3: f = &s->psiE[c][a]; break;
    case 4: f = &s->psiH[c][a]; break;
    case 5: f = &s->psiEa[c][a]; break;
    case 6: f = &s->psiHa[c][a]; break;
    default: return NULL;
    }
    for (int d = 0; d < 3; ++d) ext[d] = f->n[d];
    return f->v;
}

/* One adjoint CPML term: returns dbar and updates psibar in place. */
static double adj_pml(double tbar, double *psibar, double b, double c, double kap)
{
    const double tot = *psibar + tbar;
    *psibar = b * tot;
    return tbar / kap + c * tot;
}

/* Index of node/half-position i along a periodic axis. */
static int pw(const osim *s, int a, int i) { return s->bc[a] == OR_PERIODIC ? wrap(s, a, i) : i; }

/* Reverse of the periodic copy node n <- node 0 made after each E update. */
static void adj_fold_periodic(osim *s)
{
    for (int c = 0; c < 3; ++c) {
        ofield f = s->Ea[c];
        for (int a = 0; a < 3; ++a) {
            if (a == c || s->bc[a] != OR_PERIODIC) continue;
            int n = s->n[a];
            for (int i = 0; i < f.n[0]; ++i)
                for (int j = 0; j < f.n[1]; ++j)
                    for (int k = 0; k < f.n[2]; ++k) {
                        int id[3] = {i, j, k};
                        if (id[a] != n) continue;
                        double v = AT(f, i, j, k);
                        AT(f, i, j, k) = 0.0;
                        id[a] = 0;
                        AT(f, id[0], id[1], id[2]) += v;
                    }
        }
    }
}

/*
 * Reverse of steps 3+4 (Eq. 6 then Eq. 8).  En, Jn: E^n and J^{n-1/2} of the
 * forward run (same layout as the E arrays, components back to back); gca,
 * gcb accumulate dL/dca and dL/dcb per edge (NULL: no gradient).
 */
static void adj_update_E(osim *s, const double *En, const double *Jn, double *gca, double *gcb)
{
    const double ce = s->dt / (OR_EPS0 * s->dx);
    const double cj = s->dt / OR_EPS0;
    size_t off = 0;
    for (int c = 0; c < 3; ++c) {
        ofield E = s->Ea[c];
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;  /* curl: + d/d(a1) of H(a2), - d/d(a2) of H(a1) */
        for (int i = 0; i < E.n[0]; ++i)
            for (int j = 0; j < E.n[1]; ++j)
                for (int k = 0; k < E.n[2]; ++k) {
                    int id[3] = {i, j, k};
                    if (!e_node_updated(s, a1, id[a1]) || !e_node_updated(s, a2, id[a2])) continue;
                    const double ab = AT(E, i, j, k);
                    /* + (H_a2(id) - H_a2(id - e_a1)) */
                    double t1 = ce * ab;
                    if (s->lE[a1][id[a1]])
                        t1 = adj_pml(t1, &AT(s->psiEa[c][a1], i, j, k), s->bE[a1][id[a1]], s->cE[a1][id[a1]], s->kE[a1][id[a1]]);
                    /* - (H_a1(id) - H_a1(id - e_a2)) */
                    double t2 = -ce * ab;
                    if (s->lE[a2][id[a2]])
                        t2 = adj_pml(t2, &AT(s->psiEa[c][a2], i, j, k), s->bE[a2][id[a2]], s->cE[a2][id[a2]], s->kE[a2][id[a2]]);
                    int m1[3] = {i, j, k}, m2[3] = {i, j, k};
                    m1[a1] = pw(s, a1, id[a1] - 1);
                    m2[a2] = pw(s, a2, id[a2] - 1);
                    AT(s->Ha[a2], i, j, k) += t1;
                    AT(s->Ha[a2], m1[0], m1[1], m1[2]) -= t1;
                    AT(s->Ha[a1], i, j, k) += t2;
                    AT(s->Ha[a1], m2[0], m2[1], m2[2]) -= t2;
                    /* J^{n+1/2} enters as - (dt/eps0) J; J^{n+1/2} = ca J^{n-1/2} + cb E^n */
                    const double jt = AT(s->Ja[c], i, j, k) - cj * ab;
                    const size_t q = off + ((size_t)i * E.n[1] + j) * E.n[2] + k;
                    if (gca) {
                        gca[q] += jt * Jn[q];
                        gcb[q] += jt * En[q];
                    }
                    AT(s->Ja[c], i, j, k) = AT(s->ca[c], i, j, k) * jt;
                    AT(E, i, j, k) = ab + AT(s->cb[c], i, j, k) * jt;
                }
        off += fsize(&s->E[c]);
    }
}

/* Reverse of step 1: H^{n+1/2} = H^{n-1/2} - (dt/mu0) curl E^n. */
static void adj_update_H(osim *s)
{
    const double ch = s->dt / (OR_MU0 * s->dx);
    for (int c = 0; c < 3; ++c) {
        ofield H = s->Ha[c];
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;  /* curl: + d/d(a1) of E(a2), - d/d(a2) of E(a1) */
        for (int i = 0; i < H.n[0]; ++i)
            for (int j = 0; j < H.n[1]; ++j)
                for (int k = 0; k < H.n[2]; ++k) {
                    int id[3] = {i, j, k};
                    const double ab = AT(H, i, j, k);
                    /* H -= ch ( (E_a2(id + e_a1) - E_a2(id)) - (E_a1(id + e_a2) - E_a1(id)) ) */
                    double t1 = -ch * ab;
                    if (s->lH[a1][id[a1]])
                        t1 = adj_pml(t1, &AT(s->psiHa[c][a1], i, j, k), s->bH[a1][id[a1]], s->cH[a1][id[a1]], s->kH[a1][id[a1]]);
                    double t2 = ch * ab;
                    if (s->lH[a2][id[a2]])
                        t2 = adj_pml(t2, &AT(s->psiHa[c][a2], i, j, k), s->bH[a2][id[a2]], s->cH[a2][id[a2]], s->kH[a2][id[a2]]);
                    int p1[3] = {i, j, k}, p2[3] = {i, j, k};
                    p1[a1] += 1;
                    p2[a2] += 1;
                    AT(s->Ea[a2], p1[0], p1[1], p1[2]) += t1;
                    AT(s->Ea[a2], i, j, k) -= t1;
                    AT(s->Ea[a1], p2[0], p2[1], p2[2]) += t2;
                    AT(s->Ea[a1], i, j, k) -= t2;
                }
    }
}

/* Transpose of one field step (J_b fixed, no probes, no gradient). */
void osim_adj_step(osim *s)
{
    adj_alloc(s);
    adj_fold_periodic(s);
    adj_update_E(s, NULL, NULL, NULL, NULL);
    adj_update_H(s);
}

/* Run n steps from the current state and write J_b^{n+1/2} of each (n x jb_size). */
void osim_run_record_jb(osim *s, long n, double *out)
{
    const size_t nj = (size_t)osim_jb_size(s);
    for (long it = 0; it < n; ++it) {
        update_H(s);
        source_step(s);
        jb_save(s, out + (size_t)it * nj);
        update_E(s);
        s->step++;
        sample_probes(s);
    }
}

/*
 * Forward N steps from the current state (particles, or the prescribed
 * current), then the adjoint back to the start; L and the gradients (per
 * cell, C order like the maps) with the bunch current held at what the
 * forward run produced.  Needs at least one probe.
 */
void osim_grad(osim *s, long N, double w0, double *L, double *g_wp, double *g_gamma)
{
    const int np = s->nprobe;
    size_t nE = 0;
    for (int c = 0; c < 3; ++c) nE += fsize(&s->E[c]);
    double *hE = malloc(sizeof(double) * nE * (size_t)(N > 0 ? N : 1));
    double *hJ = malloc(sizeof(double) * nE * (size_t)(N > 0 ? N : 1));
    double *Fr = calloc((size_t)np + 1, sizeof(double)), *Fi = calloc((size_t)np + 1, sizeof(double));
    const long step0 = s->step;
    for (long n = 0; n < N; ++n) {
        size_t o = 0;
        for (int c = 0; c < 3; ++c) {
            memcpy(hE + (size_t)n * nE + o, s->E[c].v, fsize(&s->E[c]) * sizeof(double));
            memcpy(hJ + (size_t)n * nE + o, s->J[c].v, fsize(&s->J[c]) * sizeof(double));
            o += fsize(&s->E[c]);
        }
        osim_step(s, 1);
        const double th = w0 * (double)s->step * s->dt;
        for (int p = 0; p < np; ++p) {
            const double ez = AT(s->E[2], s->pijk[3 * p], s->pijk[3 * p + 1], s->pijk[3 * p + 2]);
            Fr[p] += s->dt * ez * cos(th);
            Fi[p] -= s->dt * ez * sin(th);
        }
    }
    double l = 0.0;
    for (int p = 0; p < np; ++p) l += Fr[p] * Fr[p] + Fi[p] * Fi[p];
    *L = l;

    osim_adj_zero(s);
    double *gca = calloc(nE, sizeof(double)), *gcb = calloc(nE, sizeof(double));
    for (long n = N - 1; n >= 0; --n) {
        /* dL/dEz_p^{n+1} = 2 dt (Re F cos th - Im F sin th) */
        const double th = w0 * (double)(step0 + n + 1) * s->dt;
        for (int p = 0; p < np; ++p)
            AT(s->Ea[2], s->pijk[3 * p], s->pijk[3 * p + 1], s->pijk[3 * p + 2]) +=
                2.0 * s->dt * (Fr[p] * cos(th) - Fi[p] * sin(th));
        adj_fold_periodic(s);
        adj_update_E(s, hE + (size_t)n * nE, hJ + (size_t)n * nE, gca, gcb);
        adj_update_H(s);
    }
    /* chain rule to (wp, gamma) of the owning cell (lower-corner rule) */
    memset(g_wp, 0, sizeof(double) * (size_t)s->n[0] * s->n[1] * s->n[2]);
    memset(g_gamma, 0, sizeof(double) * (size_t)s->n[0] * s->n[1] * s->n[2]);
    const double dt = s->dt;
    size_t off = 0;
    for (int c = 0; c < 3; ++c) {
        ofield E = s->E[c];
        for (int i = 0; i < E.n[0]; ++i)
            for (int j = 0; j < E.n[1]; ++j)
                for (int k = 0; k < E.n[2]; ++k) {
                    const size_t q = off + ((size_t)i * E.n[1] + j) * E.n[2] + k;
                    if (gca[q] == 0.0 && gcb[q] == 0.0) continue;
                    const int ci = clampi(i, s->n[0]), cj = clampi(j, s->n[1]), ck = clampi(k, s->n[2]);
                    const size_t m = cidx(s, ci, cj, ck);
                    const double wp = s->wp_map[m], g = s->gamma_map[m];
                    const double den = 2.0 + g * dt;
                    /* derivatives of the Eq. 6 coefficients */
                    const double dca_dg = -4.0 * dt / (den * den);
                    const double dcb_dwp = 4.0 * dt * OR_EPS0 * wp / den;
                    const double dcb_dg = -2.0 * dt * dt * OR_EPS0 * wp * wp / (den * den);
                    g_wp[m] += gcb[q] * dcb_dwp;
                    g_gamma[m] += gca[q] * dca_dg + gcb[q] * dcb_dg;
                }
        off += fsize(&E);
    }
    free(gca);
    free(gcb);
    free(hE);
    free(hJ);
    free(Fr);
    free(Fi);
}
