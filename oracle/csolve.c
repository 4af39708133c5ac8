/*
 * csolve.c -- plain C, FP64 matrix-free oracle of the semilinear lens solve.
 * TEST INFRASTRUCTURE ONLY: used by the test-suite (cross-checked against the
 * numpy oracle) and timed as the CPU baseline.  The GPU library never links it.
 *
 * Follows Rogers & Fiege (2011):
 *   thin-lens mapping (Eq. 1), SIE deflection with s = 0 (Eqs. 10-11), plus
 *   external shear (not in the paper); subpixel tracing and averaging
 *   (Sec. 2.2); bilinear source interpolation (Sec. 2.1); zero-padded PSF
 *   convolution B and its correlation B^T (Sec. 2.2); regularised normal
 *   equations (L^T B^T B L + lambda H^T H) s = L^T B^T d (Eq. 7 with x0 = 0,
 *   Eq. 13-14), solved by CG from a blank source (Sec. 2.2); chi^2 (Eq. 4) and
 *   reg = ||H s||^2 (Sec. 2.6).
 *
 * Conventions (identical to the numpy oracle): pixel centres
 * ((c-(nx-1)/2)p, (r-(ny-1)/2)p); subpixel offsets ((a+1/2)/n-1/2)p; source
 * nodes at -R + c h, h = 2R/(ns-1); inside iff 0<=u,v<=ns-1; c0 =
 * min(floor u, ns-2); weights divided by n^2; curvature H = Dirichlet second
 * differences along x and y.  One OpenMP thread per member.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ST_OK = 0, ST_MAXIT = 1, ST_EMPTY = 2, ST_BREAKDOWN = 3 };

typedef struct {
    int nx, ny, nsub, ns, K, reg;
    double pix, R;
    const double *psf, *d;
    int nsp;          /* subpixels per pixel */
    int *idx;         /* [J*nsp] node (r0*ns+c0) or -1 */
    double *fx, *fy;  /* [J*nsp] */
    double *img, *img2;
} member_t;

static void trace_member(member_t *m, const double *lens) {
    double b = lens[0], q = lens[1], pa = lens[2], g = lens[3], gpa = lens[4];
    double x0 = lens[5], y0 = lens[6];
    double cp = cos(pa), sp = sin(pa);
    double k = sqrt(fmax(0.0, 1.0 - q * q));
    double g1 = g * cos(2.0 * gpa), g2 = g * sin(2.0 * gpa);
    double h = 2.0 * m->R / (m->ns - 1);
    int n = m->nsub;
    for (int r = 0; r < m->ny; ++r)
        for (int c = 0; c < m->nx; ++c)
            for (int sr = 0; sr < n; ++sr)
                for (int sc = 0; sc < n; ++sc) {
                    double x = (c - (m->nx - 1) / 2.0) * m->pix + ((sc + 0.5) / n - 0.5) * m->pix;
                    double y = (r - (m->ny - 1) / 2.0) * m->pix + ((sr + 0.5) / n - 0.5) * m->pix;
                    double dx = x - x0, dy = y - y0;
                    double xp = cp * dx + sp * dy, yp = -sp * dx + cp * dy;
                    double psi = sqrt(q * q * xp * xp + yp * yp);
                    double axp = 0.0, ayp = 0.0;
                    if (psi > 0.0) {
                        if (k < 1e-4) {
                            axp = b * q * xp / psi;
                            ayp = b * q * yp / psi;
                        } else {
                            axp = (b * q / k) * atan(k * xp / psi);
                            ayp = (b * q / k) * atanh(k * yp / psi);
                        }
                    }
                    double ax = cp * axp - sp * ayp, ay = sp * axp + cp * ayp;
                    double bx = x - ax - (g1 * dx + g2 * dy);
                    double by = y - ay - (g2 * dx - g1 * dy);
                    double u = (bx + m->R) / h, v = (by + m->R) / h;
                    size_t t = ((size_t)(r * m->nx + c)) * m->nsp + sr * n + sc;
                    if (u >= 0.0 && u <= m->ns - 1 && v >= 0.0 && v <= m->ns - 1) {
                        int c0 = (int)floor(u), r0 = (int)floor(v);
                        if (c0 > m->ns - 2) c0 = m->ns - 2;
                        if (r0 > m->ns - 2) r0 = m->ns - 2;
                        m->idx[t] = r0 * m->ns + c0;
                        m->fx[t] = u - c0;
                        m->fy[t] = v - r0;
                    } else {
                        m->idx[t] = -1;
                        m->fx[t] = m->fy[t] = 0.0;
                    }
                }
}

static void op_L(const member_t *m, const double *s, double *img) {
    int J = m->nx * m->ny, ns = m->ns;
    double inv = 1.0 / (double)m->nsp;
    for (int j = 0; j < J; ++j) {
        double acc = 0.0;
        for (int k = 0; k < m->nsp; ++k) {
            size_t t = (size_t)j * m->nsp + k;
            int i = m->idx[t];
            if (i < 0) continue;
            double fx = m->fx[t], fy = m->fy[t];
            acc += (1 - fx) * (1 - fy) * s[i] + fx * (1 - fy) * s[i + 1] +
                   (1 - fx) * fy * s[i + ns] + fx * fy * s[i + ns + 1];
        }
        img[j] = acc * inv;
    }
}

static void op_LT(const member_t *m, const double *img, double *s) {
    int J = m->nx * m->ny, ns = m->ns;
    double inv = 1.0 / (double)m->nsp;
    memset(s, 0, sizeof(double) * ns * ns);
    for (int j = 0; j < J; ++j) {
        double v = img[j] * inv;
        for (int k = 0; k < m->nsp; ++k) {
            size_t t = (size_t)j * m->nsp + k;
            int i = m->idx[t];
            if (i < 0) continue;
            double fx = m->fx[t], fy = m->fy[t];
            s[i] += (1 - fx) * (1 - fy) * v;
            s[i + 1] += fx * (1 - fy) * v;
            s[i + ns] += (1 - fx) * fy * v;
            s[i + ns + 1] += fx * fy * v;
        }
    }
}

/* transpose=0: convolution B; transpose=1: correlation B^T */
static void op_B(const member_t *m, const double *in, double *out, int transpose) {
    int K = m->K, ck = (K - 1) / 2, nx = m->nx, ny = m->ny;
    for (int r = 0; r < ny; ++r)
        for (int c = 0; c < nx; ++c) {
            double acc = 0.0;
            for (int a = 0; a < K; ++a) {
                int rr = transpose ? r + a - ck : r - a + ck;
                if (rr < 0 || rr >= ny) continue;
                for (int b = 0; b < K; ++b) {
                    int cc = transpose ? c + b - ck : c - b + ck;
                    if (cc < 0 || cc >= nx) continue;
                    acc += m->psf[a * K + b] * in[rr * nx + cc];
                }
            }
            out[r * nx + c] = acc;
        }
}

static double node(const double *s, int ns, int r, int c) {
    return (r < 0 || c < 0 || r >= ns || c >= ns) ? 0.0 : s[r * ns + c];
}

static double d2x(const double *s, int ns, int r, int c) {
    if (r < 0 || c < 0 || r >= ns || c >= ns) return 0.0;
    return node(s, ns, r, c - 1) - 2.0 * node(s, ns, r, c) + node(s, ns, r, c + 1);
}

static double d2y(const double *s, int ns, int r, int c) {
    if (r < 0 || c < 0 || r >= ns || c >= ns) return 0.0;
    return node(s, ns, r - 1, c) - 2.0 * node(s, ns, r, c) + node(s, ns, r + 1, c);
}

/* out = H^T H s */
static void op_HtH(int ns, int kind, const double *s, double *out) {
    int I = ns * ns;
    if (kind == 0) {
        memcpy(out, s, sizeof(double) * I);
        return;
    }
    for (int r = 0; r < ns; ++r)
        for (int c = 0; c < ns; ++c)
            out[r * ns + c] = d2x(s, ns, r, c - 1) - 2.0 * d2x(s, ns, r, c) + d2x(s, ns, r, c + 1) +
                              d2y(s, ns, r - 1, c) - 2.0 * d2y(s, ns, r, c) + d2y(s, ns, r + 1, c);
}

static double reg_term(int ns, int kind, const double *s) {
    double acc = 0.0;
    if (kind == 0) {
        for (int i = 0; i < ns * ns; ++i) acc += s[i] * s[i];
        return acc;
    }
    for (int r = 0; r < ns; ++r)
        for (int c = 0; c < ns; ++c) {
            double a = d2x(s, ns, r, c), b = d2y(s, ns, r, c);
            acc += a * a + b * b;
        }
    return acc;
}

static double dot(const double *a, const double *b, int n) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += a[i] * b[i];
    return acc;
}

/* q = L^T B^T B L p + lambda H^T H p */
static void normal_op(member_t *m, double lam, const double *p, double *q, double *tmp) {
    int I = m->ns * m->ns;
    op_L(m, p, m->img);
    op_B(m, m->img, m->img2, 0);
    op_B(m, m->img2, m->img, 1);
    op_LT(m, m->img, q);
    op_HtH(m->ns, m->reg, p, tmp);
    for (int i = 0; i < I; ++i) q[i] += lam * tmp[i];
}

int oracle_eval(int n_members, const double *lens, const int *ns_arr, double half_width, int nx,
                int ny, double pix, int nsub, const double *d, double sigma, const double *psf,
                int K, int reg_kind, const double *lambdas, int n_lambda, double tol, int maxit,
                double *chi2, double *reg, int *iters, int *status, double *s_out, int s_stride,
                int threads) {
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int mi = 0; mi < n_members; ++mi) {
        member_t m;
        m.nx = nx; m.ny = ny; m.nsub = nsub; m.ns = ns_arr[mi]; m.K = K; m.reg = reg_kind;
        m.pix = pix; m.R = half_width; m.psf = psf; m.d = d; m.nsp = nsub * nsub;
        int J = nx * ny, I = m.ns * m.ns;
        m.idx = (int *)malloc(sizeof(int) * (size_t)J * m.nsp);
        m.fx = (double *)malloc(sizeof(double) * (size_t)J * m.nsp);
        m.fy = (double *)malloc(sizeof(double) * (size_t)J * m.nsp);
        m.img = (double *)malloc(sizeof(double) * J);
        m.img2 = (double *)malloc(sizeof(double) * J);
        double *b = (double *)malloc(sizeof(double) * I);
        double *s = (double *)malloc(sizeof(double) * I);
        double *r = (double *)malloc(sizeof(double) * I);
        double *p = (double *)malloc(sizeof(double) * I);
        double *q = (double *)malloc(sizeof(double) * I);
        double *tmp = (double *)malloc(sizeof(double) * I);
        trace_member(&m, lens + 7 * mi);
        op_B(&m, d, m.img, 1);
        op_LT(&m, m.img, b);
        double bnorm = sqrt(dot(b, b, I));
        int mx = maxit > 0 ? maxit : (10 * I > 2000 ? 10 * I : 2000);
        for (int k = 0; k < n_lambda; ++k) {
            double lam = lambdas[k];
            int st = ST_OK, it = 0;
            memset(s, 0, sizeof(double) * I);
            if (bnorm == 0.0) {
                st = ST_EMPTY;
            } else {
                memcpy(r, b, sizeof(double) * I);
                memcpy(p, b, sizeof(double) * I);
                double rr = dot(r, r, I);
                st = ST_MAXIT;
                for (it = 0; it < mx; ++it) {
                    if (sqrt(rr) <= tol * bnorm) { st = ST_OK; break; }
                    normal_op(&m, lam, p, q, tmp);
                    double pq = dot(p, q, I);
                    if (!(pq > 0.0)) { st = ST_BREAKDOWN; break; }
                    double alpha = rr / pq;
                    for (int i = 0; i < I; ++i) { s[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
                    double rn = dot(r, r, I);
                    double beta = rn / rr;
                    for (int i = 0; i < I; ++i) p[i] = r[i] + beta * p[i];
                    rr = rn;
                }
                if (st == ST_MAXIT && sqrt(rr) <= tol * bnorm) st = ST_OK;
            }
            /* chi^2 from the explicit solution */
            op_L(&m, s, m.img);
            op_B(&m, m.img, m.img2, 0);
            double c2 = 0.0;
            for (int j = 0; j < J; ++j) {
                double e = m.img2[j] - d[j];
                c2 += e * e;
            }
            size_t o = (size_t)mi * n_lambda + k;
            chi2[o] = c2 / (sigma * sigma);
            reg[o] = reg_term(m.ns, reg_kind, s);
            iters[o] = it;
            status[o] = st;
            if (s_out) memcpy(s_out + o * (size_t)s_stride, s, sizeof(double) * I);
        }
        free(m.idx); free(m.fx); free(m.fy); free(m.img); free(m.img2);
        free(b); free(s); free(r); free(p); free(q); free(tmp);
    }
    return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
