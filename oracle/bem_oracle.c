/*
 * CPU FP64 oracle for the piecewise-constant displacement-discontinuity (DD)
 * collocation operator of the paper (Sec. 3.1, "Solid mechanics": traction
 * hypersingular BIE, piecewise-constant DD per element, collocation at the
 * element centroid, integrals taken before the limit so they stay regular).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * Two independent derivations of the same coefficient live here:
 *   (1) coplanar closed form for rectangles sharing one plane and one frame,
 *       obtained from the Fourier symbol of the planar-crack traction
 *       operator (corner antiderivatives of the finite-part integrals);
 *   (2) any flat polygon, any receiver point: the stress of a uniform DD on
 *       a flat polygon equals that of the dislocation loop along its
 *       boundary with Burgers vector equal to the DD (Volterra), evaluated
 *       with the Peach-Koehler line integral by adaptive Gauss-Legendre
 *       quadrature along each straight edge.
 * The tests pin each against the other and against closed-form solutions.
 *
 * Conventions (paper Sec. 2.2 and Sec. 3.1 "local Cartesian coordinate
 * system"): DD delta = u+ - u-, components in the element frame (s1, s2, n);
 * tractions in the receiver frame; E[a][b] = traction component a at the
 * receiver centroid due to a unit DD component b on the source element
 * (Pa/m).  The frame: s1 = unit(v1 - v0), n = unit((v1 - v0) x (v2 - v0)),
 * s2 = n x s1; centroid = vertex mean.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* small vector helpers                                                */
/* ------------------------------------------------------------------ */
static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double* a) { return sqrt(dot3(a, a)); }

/* ------------------------------------------------------------------ */
/* element geometry                                                    */
/* ------------------------------------------------------------------ */
/* frame rows: s1, s2, n.  Returns 0, or -1 for a degenerate element. */
static int element_frame(int nvpe, const double* v, double* cent, double* fr, double* area)
{
    double e1[3], e2[3], nn[3];
    for (int k = 0; k < 3; ++k) {
        cent[k] = 0.0;
        for (int q = 0; q < nvpe; ++q) cent[k] += v[3 * q + k];
        cent[k] /= nvpe;
        e1[k] = v[3 + k] - v[k];
        e2[k] = v[6 + k] - v[k];
    }
    cross3(e1, e2, nn);
    double l1 = norm3(e1), ln = norm3(nn);
    if (l1 == 0.0 || ln == 0.0) return -1;
    for (int k = 0; k < 3; ++k) {
        fr[k] = e1[k] / l1;
        fr[6 + k] = nn[k] / ln;
    }
    cross3(fr + 6, fr, fr + 3);
    /* polygon area by fan triangulation from v0 */
    double a = 0.0;
    for (int q = 1; q + 1 < nvpe; ++q) {
        double p1[3], p2[3], c[3];
        for (int k = 0; k < 3; ++k) {
            p1[k] = v[3 * q + k] - v[k];
            p2[k] = v[3 * (q + 1) + k] - v[k];
        }
        cross3(p1, p2, c);
        a += 0.5 * norm3(c);
    }
    *area = a;
    return 0;
}

int orc_frames(int nvpe, int64_t ne, const double* xyz, const int64_t* conn,
               double* cent, double* frame, double* area)
{
    for (int64_t e = 0; e < ne; ++e) {
        double v[12];
        for (int q = 0; q < nvpe; ++q)
            for (int k = 0; k < 3; ++k) v[3 * q + k] = xyz[3 * conn[e * nvpe + q] + k];
        if (element_frame(nvpe, v, cent + 3 * e, frame + 9 * e, area + e) != 0) return -1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* (1) coplanar closed form, axis-aligned rectangle                    */
/* ------------------------------------------------------------------ */
/*
 * For a receiver and a source sharing a plane and a frame, the planar-crack
 * traction operator has Fourier symbol
 *   normal:     -(G / (2 (1 - nu))) |k|
 *   tangential: -(G / 2) [ |k| delta_ab + nu / (1 - nu) k_a k_b / |k| ],
 * which in real space gives, with c0 = G / (4 pi (1 - nu)) and finite-part
 * integrals over the source of the in-plane offset (xi, zeta) = y - x:
 *   E^nn   = c0 I0
 *   E^s1s1 = c0 [(1 - 2 nu) I0 + 3 nu Ixx]
 *   E^s2s2 = c0 [(1 - 2 nu) I0 + 3 nu Izz]
 *   E^s1s2 = E^s2s1 = 3 nu c0 Ixz,  E^sn = E^ns = 0
 * with I0 = fp int r^-3, Ixx = fp int xi^2 r^-5, Izz = fp int zeta^2 r^-5,
 * Ixz = int xi zeta r^-5.  Over [xi1, xi2] x [ze1, ze2] each integral is the
 * corner sum F(xi2, ze2) - F(xi1, ze2) - F(xi2, ze1) + F(xi1, ze1) of a
 * mixed antiderivative F (d2F / dxi dze = integrand); at an interior point
 * the corner sum equals the Hadamard finite part.
 */
static double F0(double x, double z) { double r = sqrt(x * x + z * z); return -r / (x * z); }
static double Fxx(double x, double z) { double r = sqrt(x * x + z * z); return -(r / (x * z) + z / (x * r)) / 3.0; }
static double Fzz(double x, double z) { double r = sqrt(x * x + z * z); return -(r / (x * z) + x / (z * r)) / 3.0; }
static double Fxz(double x, double z) { double r = sqrt(x * x + z * z); return 1.0 / (3.0 * r); }

static double corner_sum(double (*F)(double, double), double x1, double x2, double z1, double z2)
{
    return F(x2, z2) - F(x1, z2) - F(x2, z1) + F(x1, z1);
}

void orc_coplanar_rect_block(double young, double nu, double xi1, double xi2, double ze1, double ze2,
                             double* out /* [3][3] */)
{
    double G = young / (2.0 * (1.0 + nu));
    double c0 = G / (4.0 * ORC_PI * (1.0 - nu));
    double I0 = corner_sum(F0, xi1, xi2, ze1, ze2);
    double Ixx = corner_sum(Fxx, xi1, xi2, ze1, ze2);
    double Izz = corner_sum(Fzz, xi1, xi2, ze1, ze2);
    double Ixz = corner_sum(Fxz, xi1, xi2, ze1, ze2);
    memset(out, 0, 9 * sizeof(double));
    out[0] = c0 * ((1.0 - 2.0 * nu) * I0 + 3.0 * nu * Ixx);
    out[4] = c0 * ((1.0 - 2.0 * nu) * I0 + 3.0 * nu * Izz);
    out[1] = out[3] = 3.0 * nu * c0 * Ixz;
    out[8] = c0 * I0;
}

/* ------------------------------------------------------------------ */
/* (2) Peach-Koehler loop integral                                     */
/* ------------------------------------------------------------------ */
/*
 * Stress at x of a dislocation loop C with Burgers vector b, line element
 * dx' along C, r = x - x', R = |r|, derivatives with respect to x:
 *   sig_ac = -(G / 8pi) oint b_m eps_ima d_i(lap R) dx'_c
 *            -(G / 8pi) oint b_m eps_imc d_i(lap R) dx'_a
 *            -(G / (4pi (1 - nu))) oint b_m eps_imk (d_i d_a d_c R - delta_ac d_i(lap R)) dx'_k
 * with d_i(lap R) = -2 r_i / R^3 and
 *      d_i d_a d_c R = -(delta_ia r_c + delta_ic r_a + delta_ac r_i) / R^3 + 3 r_i r_a r_c / R^5.
 * The loop runs v0 -> v1 -> ... -> v0, counter-clockwise about the source
 * normal, and b = delta = u+ - u- (global components).  With that loop sense
 * the formula holds as written: its coplanar limit is the planar-crack
 * operator of (1) (negative self-coefficient, opening under pressure), which
 * the tests check entry by entry.
 */

/*
 * The sums over the Levi-Civita symbol contract to cross products:
 *   sum_{i,m} b_m eps_ima D_i = (D x b)_a and sum_{m,k} b_m eps_imk e_k = (b x e)_i,
 * so with D = grad(lap R) = -2 r / R^3 and w = b x e:
 *   sig_ac = c1 [(D x b)_a e_c + (D x b)_c e_a]
 *          + c3 [-(w_a r_c + w_c r_a + delta_ac (w.r)) / R^3 + 3 (w.r) r_a r_c / R^5
 *                - delta_ac (w.D)],
 * c1 = -G / (8 pi), c3 = -G / (4 pi (1 - nu)).
 */
static void pk_integrand(double G, double nu, const double* x, const double* xp, const double* e,
                         const double* b, double sig[3][3])
{
    double r[3] = {x[0] - xp[0], x[1] - xp[1], x[2] - xp[2]};
    double R = norm3(r);
    double R3 = R * R * R, R5 = R3 * R * R;
    double D1[3];
    for (int i = 0; i < 3; ++i) D1[i] = -2.0 * r[i] / R3;
    double c1 = -G / (8.0 * ORC_PI);
    double c3 = -G / (4.0 * ORC_PI * (1.0 - nu));
    double Db[3], w[3];
    cross3(D1, b, Db);
    cross3(b, e, w);
    double wr = dot3(w, r), wD = dot3(w, D1);
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            double dac = (a == c) ? 1.0 : 0.0;
            double t3 = -(w[a] * r[c] + w[c] * r[a] + dac * wr) / R3 + 3.0 * wr * r[a] * r[c] / R5 - dac * wD;
            sig[a][c] = c1 * (Db[a] * e[c] + Db[c] * e[a]) + c3 * t3;
        }
}

/* block integrand along one edge: out9[a*3+b] = s_a^r . sig(b = e_b^src) . n^r */
typedef struct {
    double G, nu;
    const double* x;     /* receiver point */
    const double* fr;    /* receiver frame rows s1,s2,n */
    const double* fs;    /* source frame rows s1,s2,n (DD components) */
    double p0[3], e[3];  /* edge start and unit tangent */
} edge_ctx;

static void edge_integrand(const edge_ctx* c, double s, double* out9)
{
    double xp[3];
    for (int k = 0; k < 3; ++k) xp[k] = c->p0[k] + s * c->e[k];
    for (int bb = 0; bb < 3; ++bb) {
        double sig[3][3];
        pk_integrand(c->G, c->nu, c->x, xp, c->e, c->fs + 3 * bb, sig);
        double t[3];
        for (int a = 0; a < 3; ++a) t[a] = sig[a][0] * c->fr[6] + sig[a][1] * c->fr[7] + sig[a][2] * c->fr[8];
        for (int a = 0; a < 3; ++a) out9[3 * a + bb] = dot3(c->fr + 3 * a, t);
    }
}

/* Gauss-Legendre nodes on [-1, 1] by Newton iteration on P_n */
#define GL_N 8
static double gl_x[GL_N], gl_w[GL_N];
static int gl_ready = 0;
static void gl_init(void)
{
    if (gl_ready) return;
    for (int i = 0; i < GL_N; ++i) {
        double x = cos(ORC_PI * (i + 0.75) / (GL_N + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= GL_N; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double dp = GL_N * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= GL_N; ++k) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = GL_N * (x * p1 - p0) / (x * x - 1.0);
        gl_x[i] = x;
        gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    gl_ready = 1;
}

static void gl_rule(const edge_ctx* c, double a, double b, double* out9)
{
    double mid = 0.5 * (a + b), half = 0.5 * (b - a);
    for (int k = 0; k < 9; ++k) out9[k] = 0.0;
    for (int i = 0; i < GL_N; ++i) {
        double f[9];
        edge_integrand(c, mid + half * gl_x[i], f);
        for (int k = 0; k < 9; ++k) out9[k] += half * gl_w[i] * f[k];
    }
}

static double norm9(const double* v)
{
    double s = 0.0;
    for (int k = 0; k < 9; ++k) s += v[k] * v[k];
    return sqrt(s);
}

/* adaptive bisection: accept when the two-half estimate agrees with the whole */
static void gl_adapt(const edge_ctx* c, double a, double b, const double* whole, double tol, int depth,
                     double* out9)
{
    double m = 0.5 * (a + b), left[9], right[9], two[9];
    gl_rule(c, a, m, left);
    gl_rule(c, m, b, right);
    for (int k = 0; k < 9; ++k) two[k] = left[k] + right[k];
    double diff[9];
    for (int k = 0; k < 9; ++k) diff[k] = two[k] - whole[k];
    if (depth >= 40 || norm9(diff) <= tol) {
        for (int k = 0; k < 9; ++k) out9[k] += two[k];
        return;
    }
    gl_adapt(c, a, m, left, 0.5 * tol, depth + 1, out9);
    gl_adapt(c, m, b, right, 0.5 * tol, depth + 1, out9);
}

/*
 * Traction block at receiver point xr (frame fr) due to unit DD components
 * (in source frame fs) on the flat polygon vsrc[nvs][3].  rtol is relative
 * to the magnitude of each edge's contribution.
 */
void orc_pk_block(double young, double nu, const double* xr, const double* fr, int nvs,
                  const double* vsrc, const double* fs, double rtol, double* out /* [3][3] */)
{
    gl_init();
    double G = young / (2.0 * (1.0 + nu));
    for (int k = 0; k < 9; ++k) out[k] = 0.0;
    for (int q = 0; q < nvs; ++q) {
        const double* a = vsrc + 3 * q;
        const double* b = vsrc + 3 * ((q + 1) % nvs);
        edge_ctx c;
        c.G = G;
        c.nu = nu;
        c.x = xr;
        c.fr = fr;
        c.fs = fs;
        double d[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        double L = norm3(d);
        for (int k = 0; k < 3; ++k) {
            c.p0[k] = a[k];
            c.e[k] = d[k] / L;
        }
        double whole[9], acc[9] = {0};
        gl_rule(&c, 0.0, L, whole);
        double tol = rtol * (norm9(whole) + 1e-300);
        gl_adapt(&c, 0.0, L, whole, tol, 0, acc);
        for (int k = 0; k < 9; ++k) out[k] += acc[k];
    }
}

/* ------------------------------------------------------------------ */
/* assembly of exact blocks                                            */
/* ------------------------------------------------------------------ */
typedef struct {
    int nvpe;
    const double* xyz;
    const int64_t* conn;
    double* cent;
    double* frame;
    double* area;
} mesh_view;

/* coplanar closed form applies: both rectangles, identical frames, same plane */
static int coplanar_same_frame(const mesh_view* m, int64_t i, int64_t j)
{
    if (m->nvpe != 4) return 0;
    const double* fi = m->frame + 9 * i;
    const double* fj = m->frame + 9 * j;
    for (int k = 0; k < 9; ++k)
        if (fabs(fi[k] - fj[k]) > 1e-12) return 0;
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = m->cent[3 * j + k] - m->cent[3 * i + k];
    double scale = sqrt(m->area[j]) + norm3(d);
    return fabs(dot3(d, fi + 6)) <= 1e-12 * scale;
}

static void block_ij(const mesh_view* m, double young, double nu, int64_t i, int64_t j, int method, double tol,
                     double* out)
{
    if (method != 1 && coplanar_same_frame(m, i, j)) {
        /* source corners in receiver in-plane coordinates */
        const double* f = m->frame + 9 * i;
        double xmin = 1e300, xmax = -1e300, zmin = 1e300, zmax = -1e300;
        for (int q = 0; q < 4; ++q) {
            const double* v = m->xyz + 3 * m->conn[4 * j + q];
            double d[3] = {v[0] - m->cent[3 * i], v[1] - m->cent[3 * i + 1], v[2] - m->cent[3 * i + 2]};
            double xi = dot3(d, f), ze = dot3(d, f + 3);
            xmin = fmin(xmin, xi);
            xmax = fmax(xmax, xi);
            zmin = fmin(zmin, ze);
            zmax = fmax(zmax, ze);
        }
        orc_coplanar_rect_block(young, nu, xmin, xmax, zmin, zmax, out);
        return;
    }
    double v[12];
    for (int q = 0; q < m->nvpe; ++q)
        for (int k = 0; k < 3; ++k) v[3 * q + k] = m->xyz[3 * m->conn[m->nvpe * j + q] + k];
    orc_pk_block(young, nu, m->cent + 3 * i, m->frame + 9 * i, m->nvpe, v, m->frame + 9 * j, tol, out);
}

static int make_view(mesh_view* m, int nvpe, int64_t ne, const double* xyz, const int64_t* conn)
{
    m->nvpe = nvpe;
    m->xyz = xyz;
    m->conn = conn;
    m->cent = (double*)malloc(sizeof(double) * 3 * ne);
    m->frame = (double*)malloc(sizeof(double) * 9 * ne);
    m->area = (double*)malloc(sizeof(double) * ne);
    if (!m->cent || !m->frame || !m->area) return -2;
    return orc_frames(nvpe, ne, xyz, conn, m->cent, m->frame, m->area);
}

static void free_view(mesh_view* m)
{
    free(m->cent);
    free(m->frame);
    free(m->area);
}

/*
 * out[r][c][a][b] = E_{rows[r], cols[c]}^{ab}.
 * method: 0 = closed form where it applies, PK quadrature elsewhere;
 *         1 = PK quadrature everywhere.
 */
int orc_assemble(int nvpe, int64_t nv, const double* xyz, int64_t ne, const int64_t* conn, double young,
                 double nu, int64_t nr, const int64_t* rows, int64_t nc, const int64_t* cols, int method,
                 double tol, double* out)
{
    (void)nv;
    gl_init();
    mesh_view m;
    int st = make_view(&m, nvpe, ne, xyz, conn);
    if (st != 0) {
        free_view(&m);
        return st;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t r = 0; r < nr; ++r)
        for (int64_t c = 0; c < nc; ++c) block_ij(&m, young, nu, rows[r], cols[c], method, tol, out + 9 * (r * nc + c));
    free_view(&m);
    return 0;
}

/*
 * Exact rows times a block of vectors without storing the rows:
 *   Y[k][3 r + a] = sum_j sum_b E_{rows[r], j}^{ab} X[k][3 j + b]
 * X is [nrhs][3 ne], Y is [nrhs][3 nr].
 */
int orc_rows_matvec(int nvpe, int64_t nv, const double* xyz, int64_t ne, const int64_t* conn, double young,
                    double nu, int64_t nr, const int64_t* rows, int nrhs, const double* X, double* Y, int method,
                    double tol)
{
    (void)nv;
    gl_init();
    mesh_view m;
    int st = make_view(&m, nvpe, ne, xyz, conn);
    if (st != 0) {
        free_view(&m);
        return st;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nr; ++r) {
        double* acc = (double*)calloc((size_t)3 * nrhs, sizeof(double));
        for (int64_t j = 0; j < ne; ++j) {
            double blk[9];
            block_ij(&m, young, nu, rows[r], j, method, tol, blk);
            for (int k = 0; k < nrhs; ++k) {
                const double* x = X + (size_t)k * 3 * ne + 3 * j;
                for (int a = 0; a < 3; ++a)
                    acc[3 * k + a] += blk[3 * a] * x[0] + blk[3 * a + 1] * x[1] + blk[3 * a + 2] * x[2];
            }
        }
        for (int k = 0; k < nrhs; ++k)
            for (int a = 0; a < 3; ++a) Y[(size_t)k * 3 * nr + 3 * r + a] = acc[3 * k + a];
        free(acc);
    }
    free_view(&m);
    return 0;
}

/* ------------------------------------------------------------------ */
/* (3) uniform grids: exact product by Toeplitz summation              */
/* ------------------------------------------------------------------ */
/*
 * A uniform grid of nx x ny rectangles of sides h (first in-plane axis) and
 * hy, all in one plane and one frame, element e = i + nx j centred at
 * (i h, j hy) in that frame.  The coefficient between receiver (i, j) and
 * source (k, l) depends only on the offset (k - i, l - j): it is the coplanar
 * closed form (1) for the source rectangle [di h - h/2, di h + h/2] x
 * [dj hy - hy/2, dj hy + hy/2] seen from the receiver centroid.  So the whole
 * operator is the table of the (2 nx - 1)(2 ny - 1) offsets, and E X is a
 * direct sum over all (receiver, source) pairs of that table.
 *
 * table[(dj + ny - 1)][(di + nx - 1)][a][b], di in [-(nx-1), nx-1], dj likewise.
 */
void orc_grid_table(double young, double nu, int nx, int ny, double h, double hy, double* table)
{
    const int64_t wx = 2 * (int64_t)nx - 1, wy = 2 * (int64_t)ny - 1;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < wx * wy; ++q) {
        const double di = (double)(q % wx - (nx - 1)), dj = (double)(q / wx - (ny - 1));
        orc_coplanar_rect_block(young, nu, di * h - 0.5 * h, di * h + 0.5 * h, dj * hy - 0.5 * hy,
                                dj * hy + 0.5 * hy, table + 9 * q);
    }
}

/*
 * Y[c][3 e + a] = sum over sources s = k + nx l and b of
 *     table[l - j][k - i][a][b] X[c][3 s + b],  receiver e = i + nx j.
 * X, Y are [nrhs][3 nx ny].  Direct summation over every pair, one receiver
 * per loop iteration (rows in parallel).
 */
int orc_grid_matvec(int nx, int ny, const double* table, int nrhs, const double* X, double* Y)
{
    const int64_t ne = (int64_t)nx * ny, wx = 2 * (int64_t)nx - 1;
    /* X transposed to [element][column][component] so each source is contiguous */
    double* xt = (double*)malloc(sizeof(double) * 3 * (size_t)nrhs * ne);
    if (!xt) return -2;
    for (int c = 0; c < nrhs; ++c)
        for (int64_t s = 0; s < ne; ++s)
            for (int b = 0; b < 3; ++b) xt[(s * nrhs + c) * 3 + b] = X[(size_t)c * 3 * ne + 3 * s + b];
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t e = 0; e < ne; ++e) {
        const int64_t i = e % nx, j = e / nx;
        double* acc = (double*)calloc((size_t)3 * nrhs, sizeof(double));
        if (!acc) {
            fail = 1;
            continue;
        }
        for (int64_t l = 0; l < ny; ++l)
            for (int64_t k = 0; k < nx; ++k) {
                const double* K = table + 9 * ((l - j + ny - 1) * wx + (k - i + nx - 1));
                const double* x = xt + (l * nx + k) * nrhs * 3;
                for (int c = 0; c < nrhs; ++c)
                    for (int a = 0; a < 3; ++a)
                        acc[3 * c + a] += K[3 * a] * x[3 * c] + K[3 * a + 1] * x[3 * c + 1] + K[3 * a + 2] * x[3 * c + 2];
            }
        for (int c = 0; c < nrhs; ++c)
            for (int a = 0; a < 3; ++a) Y[(size_t)c * 3 * ne + 3 * e + a] = acc[3 * c + a];
        free(acc);
    }
    free(xt);
    return fail ? -2 : 0;
}
