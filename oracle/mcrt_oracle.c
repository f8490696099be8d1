/*
 * CPU oracle: forward Monte Carlo with local estimation, and the surrogate
 * gradient.  TEST INFRASTRUCTURE ONLY (see mcrt_oracle.h).  Plain C, FP64,
 * single thread, no blocking and no reordering beyond the paper's steps.
 *
 * Paper: Holodovsky, Schechner, Levin, Levis, Aides, "In-situ
 * multi-scattering tomography", arXiv 1512.02110.  Section, equation and
 * step references below are to that paper.
 *
 * Readings where the paper is silent or garbled (each is listed in the
 * design notes of the repository):
 *  - Eq. (thetaHG) is used with the square on (1-g^2)/(1-g+2gu) restored.
 *  - Uniforms: u = ((x >> 9) + 1/2) 2^-23 from one 32-bit Philox4x32-10 word,
 *    an open interval, exact in FP32 and FP64.
 *  - Photons enter through the top face only, uniformly (Sec. 2.1.2 step i);
 *    all faces are open (step iii).
 *  - Russian roulette (step v, "following Iwabuchi"): after w <- albedo*w,
 *    if w < w_rr the photon survives with probability w/w_rr and then
 *    carries w_rr.
 *  - The local estimate (Eq. fle) is made at every collision with the
 *    incoming direction and the weight before the albedo factor.
 *  - The scattered direction is built on the orthonormal basis of Duff et al.
 *    (JCGT 2017) around the incoming direction, then renormalised.
 *  - Images are radiance per unit solar irradiance: the raw sum of local
 *    estimates times mu0 * A_top / (N * Omega_p), Omega_p the pixel solid
 *    angle.
 *  - Gradient: the surrogate of Sec. 5.2 with the in-scatter field frozen.
 *    For one local estimate C_e from a collision in voxel k_e,
 *    dC_e/dbeta(m) = C_e (delta(m,k_e)/beta(k_e) - l_e(m)), the per-event
 *    form of Eqs. (Jaco1, TcofJaco1, DivTc).
 *  - Voxelised model (Sec. 3): L_c(k) takes, per collision in voxel k, the
 *    phase function at the angle between the incoming direction and the
 *    direction from the collision point to the camera centre; j_c = L_c /
 *    beta (0 where beta = 0), scaled by mu0 A_top / N like the images.  The
 *    LOS of Eq. (taoKtoc) runs from the voxel centre to the camera centre;
 *    the sub-pixel points of Eq. (PIc) are an n x n grid of cell centres of
 *    the pixel; rays and LOS parts outside the domain contribute nothing.
 */
#include "mcrt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11): 10 rounds of two 32x32->64 multiplies with the */
/* published multipliers, key bumped by the published Weyl constants.       */

static void philox_round(uint32_t x[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x[1] ^ k[0];
    uint32_t y2 = hi0 ^ x[3] ^ k[1];
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(x, k);
    }
    memcpy(out, x, sizeof(x));
}

double oracle_uniform(uint32_t x)
{
    return ((double)(x >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Draw leg `leg` of photon `pid`: counter (pid_lo, pid_hi, leg, 0), key = seed. */
static void draw(uint64_t seed, uint64_t pid, uint32_t leg, double u[4])
{
    uint32_t ctr[4] = {(uint32_t)pid, (uint32_t)(pid >> 32), leg, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    for (int i = 0; i < 4; ++i) u[i] = oracle_uniform(r[i]);
}

/* ------------------------------------------------------------------------ */
/* Phase function, Eq. (Phg), and its inverse-transform sampling,           */
/* Eq. (thetaHG) with the square restored.                                  */

double oracle_hg_phase(double g, double c)
{
    double den = 1.0 + g * g - 2.0 * g * c;
    return (1.0 - g * g) / (4.0 * ORC_PI * den * sqrt(den));
}

double oracle_hg_sample(double g, double u)
{
    double mu;
    if (g == 0.0) {
        mu = 2.0 * u - 1.0;
    } else {
        double s = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
        mu = (1.0 + g * g - s * s) / (2.0 * g);
    }
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    return mu;
}

/* Rayleigh phase function, Eq. (Pray), and the inverse-transform sampling of
 * its polar cosine, Eq. (thetaREY): mu = gamma^(1/3) - gamma^(-1/3) with
 * gamma = 4u - 2 + sqrt((4u - 2)^2 + 1), the real root of the CDF
 * (mu^3 + 3 mu + 4) / 8 = u. */
double oracle_rayleigh_phase(double c)
{
    return 3.0 / (16.0 * ORC_PI) * (1.0 + c * c);
}

double oracle_rayleigh_sample(double u)
{
    double a = 4.0 * u - 2.0;
    double gam = a + sqrt(a * a + 1.0);
    double cg = cbrt(gam);
    double mu = cg - 1.0 / cg;
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    return mu;
}

/* Particle-type draw at collision s of photon pid (air + aerosol mixture,
 * step iv): first word of counter (pid_lo, pid_hi, s, 1). */
static double draw_type(uint64_t seed, uint64_t pid, uint32_t s)
{
    uint32_t ctr[4] = {(uint32_t)pid, (uint32_t)(pid >> 32), s, 1u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    return oracle_uniform(r[0]);
}

/* New direction at polar cosine mu and azimuth phi about w_in (step vi). */
void oracle_scatter_direction(const double w[3], double mu, double phi, double out[3])
{
    double sign = copysign(1.0, w[2]);
    double a = -1.0 / (sign + w[2]);
    double b = w[0] * w[1] * a;
    double b1[3] = {1.0 + sign * w[0] * w[0] * a, sign * b, -sign * w[0]};
    double b2[3] = {b, sign + w[1] * w[1] * a, -w[1]};
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double cp = cos(phi), sp = sin(phi);
    double n2 = 0.0;
    for (int i = 0; i < 3; ++i) {
        out[i] = st * cp * b1[i] + st * sp * b2[i] + mu * w[i];
        n2 += out[i] * out[i];
    }
    double inv = 1.0 / sqrt(n2);
    for (int i = 0; i < 3; ++i) out[i] *= inv;
}

/* Solid angle of pixel (row, col): the rectangle [x1,x2] x [y1,y2] on the
 * unit-focal plane subtends F(x2,y2)-F(x1,y2)-F(x2,y1)+F(x1,y1) with
 * F(x,y) = atan(x y / sqrt(1 + x^2 + y^2)). */
static double rect_F(double x, double y)
{
    return atan(x * y / sqrt(1.0 + x * x + y * y));
}

double oracle_pixel_solid_angle(const orc_camera* cam, int row, int col)
{
    double x1 = ((double)col - cam->cx) / cam->fx, x2 = ((double)col + 1.0 - cam->cx) / cam->fx;
    double y1 = ((double)row - cam->cy) / cam->fy, y2 = ((double)row + 1.0 - cam->cy) / cam->fy;
    return rect_F(x2, y2) - rect_F(x1, y2) - rect_F(x2, y1) + rect_F(x1, y1);
}

/* ------------------------------------------------------------------------ */
/* Voxel traversal (regular tracking): the voxel sequence of a ray and the  */
/* length of the ray inside each voxel, so that tau = sum beta(m) l(m),     */
/* Eq. (taoKtoc).                                                           */

typedef struct {
    int n[3];
    double d[3];
} geom;

typedef struct {
    double o[3], w[3];
    int i[3], step[3];
    double tmax[3];  /* ray parameter of the next face crossing on each axis */
    double t;        /* ray parameter of the entry into the current voxel */
} walker;

static void walker_init(walker* wk, const geom* G, const double o[3], const double w[3], const int i[3])
{
    for (int a = 0; a < 3; ++a) {
        wk->o[a] = o[a];
        wk->w[a] = w[a];
        wk->i[a] = i[a];
        if (w[a] > 0.0) {
            wk->step[a] = 1;
            wk->tmax[a] = ((double)(i[a] + 1) * G->d[a] - o[a]) / w[a];
        } else if (w[a] < 0.0) {
            wk->step[a] = -1;
            wk->tmax[a] = ((double)i[a] * G->d[a] - o[a]) / w[a];
        } else {
            wk->step[a] = 0;
            wk->tmax[a] = INFINITY;
        }
        if (wk->tmax[a] < 0.0) wk->tmax[a] = 0.0;
    }
    wk->t = 0.0;
}

/* Axis whose face is crossed next; ties go to the lowest axis. */
static int walker_axis(const walker* wk)
{
    int a = 0;
    if (wk->tmax[1] < wk->tmax[a]) a = 1;
    if (wk->tmax[2] < wk->tmax[a]) a = 2;
    return a;
}

enum { LEFT_NONE = -1 };

/* Cross the face on axis a.  Returns LEFT_NONE while inside the domain,
 * else the ORC_FATE_{TOP,BOTTOM,SIDE} of the face through which it left. */
static int walker_cross(walker* wk, const geom* G, int a)
{
    wk->t = wk->tmax[a];
    wk->i[a] += wk->step[a];
    if (wk->i[a] < 0 || wk->i[a] >= G->n[a]) {
        if (a == 2) return wk->step[a] > 0 ? ORC_FATE_TOP : ORC_FATE_BOTTOM;
        return ORC_FATE_SIDE;
    }
    int face = wk->i[a] + (wk->step[a] > 0 ? 1 : 0);
    wk->tmax[a] = ((double)face * G->d[a] - wk->o[a]) / wk->w[a];
    return LEFT_NONE;
}

static int64_t vox_index(const geom* G, const int i[3])
{
    return (int64_t)i[0] + (int64_t)G->n[0] * ((int64_t)i[1] + (int64_t)G->n[1] * (int64_t)i[2]);
}

/* ------------------------------------------------------------------------ */

enum { MODE_RENDER = 0, MODE_FROZEN = 1, MODE_GRAD = 2, MODE_TRACE = 3, MODE_VOXEL = 4 };

typedef struct {
    geom G;
    double L[3];
    const double* beta_t;   /* extinction used to transport photons */
    const double* beta_le;  /* extinction used by the local estimates */
    int n_cams;
    const orc_camera* cams;
    int64_t* pix_off;       /* first pixel of each camera in the image vector */
    int64_t n_pix;
    const orc_params* prm;
    double w_sun[3];
    double* norm;           /* per-pixel mu0 A_top / (N Omega_p) */
    int mode;
    double* raw;            /* per-pixel sum of local estimates */
    double* acc;            /* current photon's per-pixel sum (for images_m2) */
    int64_t* touched;
    int64_t n_touched, cap_touched;
    double* m2;
    const double* dl;
    double* grad;
    double* Lc;             /* voxel model: [camera][voxel] scattered power */
    /* air + aerosol mixture (beta_t = beta_le = beta_air + beta_aer) */
    const double* beta_air; /* NULL: one constituent (aerosol) */
    const double* beta_aer; /* sigma * the aerosol field of the reference channel */
    double sig;             /* sigma: d beta_aer / d (reference aerosol field) */
    int air;                /* particle of the current collision: 1 air, 0 aerosol */
    int full;               /* full gradient: 1 summing replay, 2 depositing replay */
    double asum;            /* summing replay: sum of a over the photon's estimates */
    int any_a;              /* summing replay: some a != 0 */
    double ev_a;            /* depositing replay: sum of a over the current collision */
    double ff_dep;          /* depositing replay: free-flight deposit weight */
    orc_stats st;
    /* trace */
    orc_path* path;
    orc_event* ev;
    int32_t* evpix;
    uint32_t max_rec;
    int32_t cur_events;
    int64_t trace_slot;
} ctx;

/* Step (ii)-(iii): fly from X (in voxel vox) along w until the optical depth
 * tau_star is reached, Eqs. (taurand, MCextinct), solved exactly voxel by
 * voxel since beta is constant in a voxel.  Returns LEFT_NONE on a
 * collision (X, vox updated) or the face through which the photon left
 * (X set to the exit point). */
static int free_flight(ctx* c, double X[3], int vox[3], const double w[3], double tau_star)
{
    walker wk;
    walker_init(&wk, &c->G, X, w, vox);
    double tau = 0.0;
    for (;;) {
        int64_t k = vox_index(&c->G, wk.i);
        double b = c->beta_t[k];
        c->st.vox_free++;
        int a = walker_axis(&wk);
        double seg = wk.tmax[a] - wk.t;
        if (b > 0.0 && tau + b * seg >= tau_star) {
            double tc = wk.t + (tau_star - tau) / b;
            if (c->ff_dep != 0.0) c->grad[k] -= c->ff_dep * (tc - wk.t);
            for (int q = 0; q < 3; ++q) {
                X[q] = wk.o[q] + tc * wk.w[q];
                vox[q] = wk.i[q];
            }
            return LEFT_NONE;
        }
        if (c->ff_dep != 0.0) c->grad[k] -= c->ff_dep * seg;
        tau += b * seg;
        int left = walker_cross(&wk, &c->G, a);
        if (left != LEFT_NONE) {
            for (int q = 0; q < 3; ++q) X[q] = wk.o[q] + wk.t * wk.w[q];
            return left;
        }
    }
}

/* Optical depth from X (in voxel vox) along unit v over length r; the part
 * of the segment outside the domain contributes nothing.  When grad_a is
 * non-zero, also subtracts grad_a * l(m) from grad[m] for every voxel m. */
static double connection_tau(ctx* c, const double* beta, const double X[3], const int vox[3],
                             const double v[3], double r, double grad_a, int count)
{
    walker wk;
    walker_init(&wk, &c->G, X, v, vox);
    double tau = 0.0;
    for (;;) {
        int64_t k = vox_index(&c->G, wk.i);
        if (count) c->st.vox_conn++;
        int a = walker_axis(&wk);
        int last = wk.tmax[a] >= r;
        double tn = last ? r : wk.tmax[a];
        double l = tn - wk.t;
        tau += beta[k] * l;
        if (grad_a != 0.0) c->grad[k] -= grad_a * l;
        if (last) break;
        if (walker_cross(&wk, &c->G, a) != LEFT_NONE) break;
    }
    return tau;
}

static void tally(ctx* c, int64_t p, double C)
{
    c->raw[p] += C;
    if (c->m2) {
        if (c->acc[p] == 0.0) {
            if (c->n_touched == c->cap_touched) {
                c->cap_touched = c->cap_touched ? 2 * c->cap_touched : 1024;
                c->touched = (int64_t*)realloc(c->touched, (size_t)c->cap_touched * sizeof(int64_t));
            }
            c->touched[c->n_touched++] = p;
        }
        c->acc[p] += C;
    }
}

/* Sec. 2.1.3, Eq. (fle): at a collision at X in voxel vox, with incoming
 * direction w and packet intensity I_s = weight, add
 * albedo I_s P(angle(w, X->X_c)) exp(-tau(X->X_c)) / |X_c - X|^2 to the pixel
 * of every camera that sees X. */
static void local_estimates(ctx* c, const double X[3], const int vox[3], const double w[3],
                            double weight)
{
    const orc_params* P = c->prm;
    int64_t ke = vox_index(&c->G, vox);
    for (int ci = 0; ci < c->n_cams; ++ci) {
        const orc_camera* cam = &c->cams[ci];
        if (c->mode == MODE_TRACE && c->evpix && c->cur_events <= (int32_t)c->max_rec)
            c->evpix[(c->trace_slot + c->cur_events - 1) * c->n_cams + ci] = -1;
        double dX[3] = {X[0] - cam->pos[0], X[1] - cam->pos[1], X[2] - cam->pos[2]};
        double q[3];
        for (int i = 0; i < 3; ++i)
            q[i] = cam->R[3 * i] * dX[0] + cam->R[3 * i + 1] * dX[1] + cam->R[3 * i + 2] * dX[2];
        if (!(q[2] > 0.0)) continue;
        double u = cam->fx * q[0] / q[2] + cam->cx;
        double v = cam->fy * q[1] / q[2] + cam->cy;
        if (!(u >= 0.0 && u < (double)cam->width && v >= 0.0 && v < (double)cam->height)) continue;
        int col = (int)floor(u), row = (int)floor(v);
        double V[3] = {-dX[0], -dX[1], -dX[2]};
        double r2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
        if (r2 < 1e-12) continue;
        double r = sqrt(r2);
        double vh[3] = {V[0] / r, V[1] / r, V[2] / r};
        double cosang = w[0] * vh[0] + w[1] * vh[1] + w[2] * vh[2];
        int64_t p = c->pix_off[ci] + (int64_t)row * cam->width + col;
        c->st.le_jobs++;
        if (c->mode == MODE_TRACE) {
            if (c->evpix && c->cur_events <= (int32_t)c->max_rec)
                c->evpix[(c->trace_slot + c->cur_events - 1) * c->n_cams + ci] = row * cam->width + col;
            continue;
        }
        double tau = connection_tau(c, c->beta_le, X, vox, vh, r, 0.0, 1);
        /* Eq. (fle) with the albedo and phase function of the particle */
        double C = c->air ? weight * oracle_rayleigh_phase(cosang) * exp(-tau) / r2
                          : P->albedo * weight * oracle_hg_phase(P->g, cosang) * exp(-tau) / r2;
        if (c->mode == MODE_FROZEN) C *= c->beta_le[ke] / c->beta_t[ke];
        if (c->mode == MODE_GRAD && c->full == 1) {
            double a = c->dl[p] * c->norm[p] * C;
            c->asum += a;
            if (a != 0.0) c->any_a = 1;
        } else if (c->mode == MODE_GRAD && c->full == 2) {
            double a = c->dl[p] * c->norm[p] * C;
            c->ev_a += a;
            if (a != 0.0) connection_tau(c, c->beta_le, X, vox, vh, r, c->sig * a, 0);
        } else if (c->mode == MODE_GRAD) {
            double a = c->dl[p] * c->norm[p] * C;
            if (a != 0.0) {
                if (!c->beta_air) {
                    c->grad[ke] += a / c->beta_t[ke];
                } else if (!c->air) {
                    c->grad[ke] += c->sig * a / c->beta_aer[ke];
                }
                connection_tau(c, c->beta_le, X, vox, vh, r, c->beta_air ? c->sig * a : a, 0);
            }
        } else {
            tally(c, p, C);
        }
    }
}

/* Sec. 3.2, Eq. (Lcupdate): a collision at X in voxel vox with incoming
 * direction w and intensity I_s = weight adds albedo I_s P(angle) to
 * L_c(vox) for every camera c, the angle between w and X -> X_c. */
static void voxel_tally(ctx* c, const double X[3], const int vox[3], const double w[3], double weight)
{
    const orc_params* P = c->prm;
    int64_t k = vox_index(&c->G, vox);
    int64_t nv = (int64_t)c->G.n[0] * c->G.n[1] * c->G.n[2];
    for (int ci = 0; ci < c->n_cams; ++ci) {
        const orc_camera* cam = &c->cams[ci];
        double V[3] = {cam->pos[0] - X[0], cam->pos[1] - X[1], cam->pos[2] - X[2]};
        double r2 = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
        if (r2 < 1e-12) continue;
        double r = sqrt(r2);
        double cosang = (w[0] * V[0] + w[1] * V[1] + w[2] * V[2]) / r;
        c->Lc[(int64_t)ci * nv + k] += P->albedo * weight * oracle_hg_phase(P->g, cosang);
        c->st.le_jobs++;
    }
}

/* The photon life cycle of Sec. 2.1.2, steps (i)-(vi). */
static int trace_photon(ctx* c, uint64_t pid)
{
    const orc_params* P = c->prm;
    double u[4];
    /* (i) launch at a uniform point of the top of the domain, along w_sun */
    draw(P->seed, pid, 0u, u);
    double X[3] = {u[0] * c->L[0], u[1] * c->L[1], c->L[2]};
    int vox[3];
    for (int a = 0; a < 2; ++a) {
        int i = (int)floor(X[a] / c->G.d[a]);
        vox[a] = i < c->G.n[a] - 1 ? i : c->G.n[a] - 1;
    }
    vox[2] = c->G.n[2] - 1;
    double w[3] = {c->w_sun[0], c->w_sun[1], c->w_sun[2]};
    double weight = 1.0;
    double tau_star = -log(1.0 - u[2]); /* Eq. (taurand) */
    uint32_t s = 0;
    for (;;) {
        /* (ii)-(iii) */
        int left = free_flight(c, X, vox, w, tau_star);
        if (left != LEFT_NONE) {
            if (left == ORC_FATE_TOP) c->st.esc_top++;
            else if (left == ORC_FATE_BOTTOM) c->st.esc_bottom++;
            else c->st.esc_side++;
            if (c->path) {
                for (int q = 0; q < 3; ++q) {
                    c->path->exit_pos[q] = X[q];
                    c->path->exit_dir[q] = w[q];
                }
                c->path->exit_w = weight;
            }
            return left;
        }
        ++s;
        c->st.events++;
        c->cur_events = (int32_t)s;
        if (c->mode == MODE_TRACE && s <= c->max_rec) {
            orc_event* e = &c->ev[c->trace_slot + s - 1];
            e->x = X[0];
            e->y = X[1];
            e->z = X[2];
            e->w = weight;
            e->voxel = (int32_t)vox_index(&c->G, vox);
            e->pad_ = 0;
        }
        /* (iv) the particle: air with probability beta_air / beta in the
         * collision voxel (mixture only) */
        int64_t kc = vox_index(&c->G, vox);
        c->air = c->beta_air ? draw_type(P->seed, pid, s) < c->beta_air[kc] / c->beta_t[kc] : 0;
        /* Sec. 2.1.3: local estimate with the incoming ray and I_s (or, for
         * the voxelised model of Sec. 3, the scattered power per voxel) */
        c->ev_a = 0.0;
        if (c->mode == MODE_VOXEL)
            voxel_tally(c, X, vox, w, weight);
        else
            local_estimates(c, X, vox, w, weight);
        if (c->full == 2) {
            /* score of collision s: the estimates of this and every later
             * collision (ff_dep / sig), over the aerosol extinction of an
             * aerosol collision; then the later ones only */
            if (!c->air && c->ff_dep != 0.0) c->grad[kc] += c->ff_dep / c->beta_aer[kc];
            c->ff_dep -= c->sig * c->ev_a;
        }
        if (s >= P->max_events) {
            c->st.capped++;
            return ORC_FATE_CAP;
        }
        draw(P->seed, pid, s, u);
        /* (v) albedo (1 for air) and Russian roulette */
        if (!c->air) weight *= P->albedo;
        if (weight < P->rr_weight) {
            if (u[2] < weight / P->rr_weight) {
                weight = P->rr_weight;
            } else {
                c->st.rr_killed++;
                return ORC_FATE_RR;
            }
        }
        /* (vi) scattering angle, Eq. (thetaHG) or (thetaREY), and uniform azimuth */
        double mu = c->air ? oracle_rayleigh_sample(u[0]) : oracle_hg_sample(P->g, u[0]);
        double phi = 2.0 * ORC_PI * u[1];
        double wn[3];
        oracle_scatter_direction(w, mu, phi, wn);
        w[0] = wn[0];
        w[1] = wn[1];
        w[2] = wn[2];
        tau_star = -log(1.0 - u[3]);
    }
}

/* ------------------------------------------------------------------------ */

static int finite_pos(double x) { return isfinite(x) && x > 0.0; }

static int validate(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                    const orc_params* P)
{
    if (!grid || !beta || !cams || !P) return ORC_ERR_INVALID_ARG;
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return ORC_ERR_INVALID_ARG;
    if (!finite_pos(grid->dx) || !finite_pos(grid->dy) || !finite_pos(grid->dz)) return ORC_ERR_INVALID_ARG;
    if ((int64_t)grid->nx * grid->ny * grid->nz > 2147483647LL) return ORC_ERR_INVALID_ARG;
    if (n_cams < 1) return ORC_ERR_INVALID_ARG;
    for (int i = 0; i < n_cams; ++i) {
        const orc_camera* c = &cams[i];
        if (c->width < 1 || c->height < 1) return ORC_ERR_INVALID_ARG;
        if (!finite_pos(c->fx) || !finite_pos(c->fy) || !isfinite(c->cx) || !isfinite(c->cy))
            return ORC_ERR_INVALID_ARG;
        for (int j = 0; j < 3; ++j) if (!isfinite(c->pos[j])) return ORC_ERR_INVALID_ARG;
        for (int j = 0; j < 9; ++j) if (!isfinite(c->R[j])) return ORC_ERR_INVALID_ARG;
    }
    if (!(P->albedo >= 0.0 && P->albedo <= 1.0)) return ORC_ERR_INVALID_ARG;
    if (!(P->g > -1.0 && P->g < 1.0)) return ORC_ERR_INVALID_ARG;
    if (!(P->sun_zenith >= 0.0 && P->sun_zenith < 0.5 * ORC_PI)) return ORC_ERR_INVALID_ARG;
    if (!isfinite(P->sun_azimuth)) return ORC_ERR_INVALID_ARG;
    if (!(P->rr_weight > 0.0 && P->rr_weight <= 1.0)) return ORC_ERR_INVALID_ARG;
    if (P->max_events < 1) return ORC_ERR_INVALID_ARG;
    int64_t nv = (int64_t)grid->nx * grid->ny * grid->nz;
    for (int64_t k = 0; k < nv; ++k)
        if (!(beta[k] >= 0.0) || !isfinite(beta[k])) return ORC_ERR_INVALID_ARG;
    return ORC_OK;
}

static void ctx_setup(ctx* c, const orc_grid* grid, const double* beta_t, const double* beta_le,
                      int n_cams, const orc_camera* cams, const orc_params* P, int mode)
{
    memset(c, 0, sizeof(*c));
    c->G.n[0] = grid->nx;
    c->G.n[1] = grid->ny;
    c->G.n[2] = grid->nz;
    c->G.d[0] = grid->dx;
    c->G.d[1] = grid->dy;
    c->G.d[2] = grid->dz;
    for (int a = 0; a < 3; ++a) c->L[a] = c->G.n[a] * c->G.d[a];
    c->beta_t = beta_t;
    c->beta_le = beta_le;
    c->n_cams = n_cams;
    c->cams = cams;
    c->prm = P;
    c->mode = mode;
    /* direction towards the sun s = (sin z cos a, sin z sin a, cos z); photons travel -s */
    c->w_sun[0] = -sin(P->sun_zenith) * cos(P->sun_azimuth);
    c->w_sun[1] = -sin(P->sun_zenith) * sin(P->sun_azimuth);
    c->w_sun[2] = -cos(P->sun_zenith);
    c->pix_off = (int64_t*)malloc((size_t)(n_cams + 1) * sizeof(int64_t));
    c->pix_off[0] = 0;
    for (int i = 0; i < n_cams; ++i)
        c->pix_off[i + 1] = c->pix_off[i] + (int64_t)cams[i].width * cams[i].height;
    c->n_pix = c->pix_off[n_cams];
    /* radiance normalisation mu0 * A_top / (N * Omega_p) with unit irradiance */
    uint64_t N = P->n_photons_norm ? P->n_photons_norm : P->n_photons;
    double base = N ? cos(P->sun_zenith) * c->L[0] * c->L[1] / (double)N : 0.0;
    c->norm = (double*)malloc((size_t)c->n_pix * sizeof(double));
    for (int i = 0; i < n_cams; ++i)
        for (int row = 0; row < cams[i].height; ++row)
            for (int col = 0; col < cams[i].width; ++col)
                c->norm[c->pix_off[i] + (int64_t)row * cams[i].width + col] =
                    base / oracle_pixel_solid_angle(&cams[i], row, col);
}

static void ctx_free(ctx* c)
{
    free(c->pix_off);
    free(c->norm);
    free(c->acc);
    free(c->touched);
}

static void run_photons(ctx* c)
{
    const orc_params* P = c->prm;
    for (uint64_t n = 0; n < P->n_photons; ++n) {
        trace_photon(c, P->photon_offset + n);
        c->st.photons++;
        if (c->m2) {
            for (int64_t t = 0; t < c->n_touched; ++t) {
                int64_t p = c->touched[t];
                double y = c->acc[p] * c->norm[p];
                c->m2[p] += y * y;
                c->acc[p] = 0.0;
            }
            c->n_touched = 0;
        }
    }
}

static int render_common(const orc_grid* grid, const double* beta_t, const double* beta_le,
                         int n_cams, const orc_camera* cams, const orc_params* P,
                         double* images, double* images_m2, orc_stats* stats, int mode)
{
    int err = validate(grid, beta_t, n_cams, cams, P);
    if (err) return err;
    if (beta_le != beta_t && (err = validate(grid, beta_le, n_cams, cams, P))) return err;
    if (!images) return ORC_ERR_INVALID_ARG;
    ctx c;
    ctx_setup(&c, grid, beta_t, beta_le, n_cams, cams, P, mode);
    c.raw = images;
    memset(images, 0, (size_t)c.n_pix * sizeof(double));
    if (images_m2) {
        c.m2 = images_m2;
        memset(images_m2, 0, (size_t)c.n_pix * sizeof(double));
        c.acc = (double*)calloc((size_t)c.n_pix, sizeof(double));
    }
    run_photons(&c);
    for (int64_t p = 0; p < c.n_pix; ++p) images[p] *= c.norm[p];
    if (stats) *stats = c.st;
    ctx_free(&c);
    return ORC_OK;
}

int oracle_render(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                  const orc_params* P, double* images, double* images_m2, orc_stats* stats)
{
    return render_common(grid, beta, beta, n_cams, cams, P, images, images_m2, stats, MODE_RENDER);
}

int oracle_render_frozen(const orc_grid* grid, const double* beta_sample, const double* beta_eval,
                         int n_cams, const orc_camera* cams, const orc_params* P,
                         double* images, orc_stats* stats)
{
    return render_common(grid, beta_sample, beta_eval, n_cams, cams, P, images, NULL, stats,
                         MODE_FROZEN);
}

int oracle_grad_beta(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                     const orc_params* P, const double* dl, double* grad, orc_stats* stats)
{
    int err = validate(grid, beta, n_cams, cams, P);
    if (err) return err;
    if (!dl || !grad) return ORC_ERR_INVALID_ARG;
    ctx c;
    ctx_setup(&c, grid, beta, beta, n_cams, cams, P, MODE_GRAD);
    c.dl = dl;
    c.grad = grad;
    memset(grad, 0, (size_t)grid->nx * grid->ny * grid->nz * sizeof(double));
    run_photons(&c);
    if (stats) *stats = c.st;
    ctx_free(&c);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Air + aerosol mixture (step iv, Eqs. Pray, thetaREY, channelBeta).       */
/* Channel extinction beta = beta_air + sigma * beta_aer_ref, sigma the     */
/* aerosol cross-section of the channel over that of the reference channel. */

typedef struct {
    double* aer;  /* sigma * beta_aer_ref */
    double* tot;  /* beta_air + aer */
} mix_fields;

static int mix_setup(const orc_grid* grid, const double* beta_air, const double* beta_aer, double sigma,
                     mix_fields* F)
{
    F->aer = F->tot = NULL;
    if (!grid || !beta_air || !beta_aer || !(sigma > 0.0) || !isfinite(sigma)) return ORC_ERR_INVALID_ARG;
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return ORC_ERR_INVALID_ARG;
    int64_t nv = (int64_t)grid->nx * grid->ny * grid->nz;
    F->aer = (double*)malloc((size_t)nv * sizeof(double));
    F->tot = (double*)malloc((size_t)nv * sizeof(double));
    for (int64_t k = 0; k < nv; ++k) {
        if (!(beta_air[k] >= 0.0) || !isfinite(beta_air[k]) || !(beta_aer[k] >= 0.0) || !isfinite(beta_aer[k])) {
            free(F->aer);
            free(F->tot);
            F->aer = F->tot = NULL;
            return ORC_ERR_INVALID_ARG;
        }
        F->aer[k] = sigma * beta_aer[k];
        F->tot[k] = beta_air[k] + F->aer[k];
    }
    return ORC_OK;
}

int oracle_render_mix(const orc_grid* grid, const double* beta_air, const double* beta_aer, double sigma,
                      int n_cams, const orc_camera* cams, const orc_params* P, double* images,
                      double* images_m2, orc_stats* stats)
{
    mix_fields F;
    int err = mix_setup(grid, beta_air, beta_aer, sigma, &F);
    if (err) return err;
    err = validate(grid, F.tot, n_cams, cams, P);
    if (!err && !images) err = ORC_ERR_INVALID_ARG;
    if (!err) {
        ctx c;
        ctx_setup(&c, grid, F.tot, F.tot, n_cams, cams, P, MODE_RENDER);
        c.beta_air = beta_air;
        c.beta_aer = F.aer;
        c.sig = sigma;
        c.raw = images;
        memset(images, 0, (size_t)c.n_pix * sizeof(double));
        if (images_m2) {
            c.m2 = images_m2;
            memset(images_m2, 0, (size_t)c.n_pix * sizeof(double));
            c.acc = (double*)calloc((size_t)c.n_pix, sizeof(double));
        }
        run_photons(&c);
        for (int64_t p = 0; p < c.n_pix; ++p) images[p] *= c.norm[p];
        if (stats) *stats = c.st;
        ctx_free(&c);
    }
    free(F.aer);
    free(F.tot);
    return err;
}

/* Gradient of the loss with respect to the reference aerosol field, added
 * to grad.  For a local estimate C_e = a_e / (dl norm) from collision e of a
 * photon whose collisions are s = 1..n (free-flight legs l_s, particles t_s):
 *  - surrogate (full = 0), Sec. 5.2 with the in-scatter field frozen:
 *      a_e (delta(m,k_e) [t_e aerosol] / beta_aer(k_e) - l_e^conn(m));
 *  - full (full = 1): the derivative of the expected image, the path
 *    probability differentiated as well (score of every collision):
 *      sum_s A_s ([t_s aerosol] delta(m,k_s) / beta_aer(k_s) - l_s(m))
 *        - sum_e a_e l_e^conn(m),   A_s = sum over collisions e >= s of a_e,
 *    computed by replaying each photon twice: once for the sum of its a,
 *    once depositing with A_s = that sum minus the estimates before s.
 * Both are times sigma (chain rule to the reference field). */
int oracle_grad_mix(const orc_grid* grid, const double* beta_air, const double* beta_aer, double sigma,
                    int n_cams, const orc_camera* cams, const orc_params* P, const double* dl, int full,
                    double* grad, orc_stats* stats)
{
    mix_fields F;
    int err = mix_setup(grid, beta_air, beta_aer, sigma, &F);
    if (err) return err;
    err = validate(grid, F.tot, n_cams, cams, P);
    if (!err && (!dl || !grad)) err = ORC_ERR_INVALID_ARG;
    if (!err) {
        ctx c;
        ctx_setup(&c, grid, F.tot, F.tot, n_cams, cams, P, MODE_GRAD);
        c.beta_air = beta_air;
        c.beta_aer = F.aer;
        c.sig = sigma;
        c.dl = dl;
        c.grad = grad;
        for (uint64_t n = 0; n < P->n_photons; ++n) {
            uint64_t pid = P->photon_offset + n;
            if (!full) {
                trace_photon(&c, pid);
            } else {
                c.full = 1;
                c.asum = 0.0;
                c.any_a = 0;
                c.ff_dep = 0.0;
                trace_photon(&c, pid);
                if (c.any_a) {
                    orc_stats keep = c.st;
                    c.full = 2;
                    c.ff_dep = sigma * c.asum;
                    trace_photon(&c, pid);
                    c.st = keep;
                    c.ff_dep = 0.0;
                }
            }
            c.st.photons++;
        }
        if (stats) *stats = c.st;
        ctx_free(&c);
    }
    free(F.aer);
    free(F.tot);
    return err;
}

int oracle_trace_paths(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                       const orc_params* P, uint64_t first_pid, uint32_t count, uint32_t max_rec,
                       orc_event* events, int32_t* pix, orc_path* paths)
{
    int err = validate(grid, beta, n_cams, cams, P);
    if (err) return err;
    if ((count > 0 && max_rec > 0 && !events) || (count > 0 && !paths)) return ORC_ERR_INVALID_ARG;
    ctx c;
    ctx_setup(&c, grid, beta, beta, n_cams, cams, P, MODE_TRACE);
    c.ev = events;
    c.evpix = pix;
    c.max_rec = max_rec;
    for (uint32_t n = 0; n < count; ++n) {
        c.trace_slot = (int64_t)n * max_rec;
        c.cur_events = 0;
        memset(&paths[n], 0, sizeof(paths[n]));
        c.path = &paths[n];
        uint64_t before = c.st.events;
        int fate = trace_photon(&c, first_pid + n);
        paths[n].n_events = (int32_t)(c.st.events - before);
        paths[n].fate = fate;
    }
    ctx_free(&c);
    return ORC_OK;
}

double oracle_optical_depth(const orc_grid* grid, const double* beta, const double p0[3],
                            const double p1[3], int64_t* nvox)
{
    ctx c;
    orc_params P;
    memset(&P, 0, sizeof(P));
    memset(&c, 0, sizeof(c));
    c.G.n[0] = grid->nx;
    c.G.n[1] = grid->ny;
    c.G.n[2] = grid->nz;
    c.G.d[0] = grid->dx;
    c.G.d[1] = grid->dy;
    c.G.d[2] = grid->dz;
    for (int a = 0; a < 3; ++a) c.L[a] = c.G.n[a] * c.G.d[a];
    double D[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    double len = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
    if (nvox) *nvox = 0;
    if (!(len > 0.0)) return 0.0;
    double v[3] = {D[0] / len, D[1] / len, D[2] / len};
    /* clip the segment to the domain (slab method) */
    double t0 = 0.0, t1 = len;
    for (int a = 0; a < 3; ++a) {
        if (v[a] == 0.0) {
            if (p0[a] < 0.0 || p0[a] > c.L[a]) return 0.0;
            continue;
        }
        double ta = (0.0 - p0[a]) / v[a], tb = (c.L[a] - p0[a]) / v[a];
        if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (!(t1 > t0)) return 0.0;
    double X[3];
    int vox[3];
    for (int a = 0; a < 3; ++a) {
        X[a] = p0[a] + t0 * v[a];
        /* the voxel entered in the direction of travel */
        double f = X[a] / c.G.d[a];
        int i = (int)floor(f);
        if (v[a] < 0.0 && f == floor(f)) i -= 1;
        if (i < 0) i = 0;
        if (i > c.G.n[a] - 1) i = c.G.n[a] - 1;
        vox[a] = i;
    }
    double tau = connection_tau(&c, beta, X, vox, v, t1 - t0, 0.0, 1);
    if (nvox) *nvox = (int64_t)c.st.vox_conn;
    return tau;
}

/* ------------------------------------------------------------------------ */
/* Voxelised forward model, Sec. 3.                                         */

/* The voxels of the segment p0 + t v, 0 <= t <= tmax (v unit), that lie in
 * the domain, with the length of the segment inside each: k[i], l[i] for
 * i < return value (at most cap).  The segment is clipped to the domain box
 * first (slab method); the walk starts in the voxel entered along v. */
static int segment_voxels(const geom* G, const double p0[3], const double v[3], double tmax,
                          int64_t* ks, double* ls, int cap)
{
    double L[3] = {G->n[0] * G->d[0], G->n[1] * G->d[1], G->n[2] * G->d[2]};
    double t0 = 0.0, t1 = tmax;
    for (int a = 0; a < 3; ++a) {
        if (v[a] == 0.0) {
            if (p0[a] < 0.0 || p0[a] > L[a]) return 0;
            continue;
        }
        double ta = (0.0 - p0[a]) / v[a], tb = (L[a] - p0[a]) / v[a];
        if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    if (!(t1 > t0)) return 0;
    double X[3];
    int vox[3];
    for (int a = 0; a < 3; ++a) {
        X[a] = p0[a] + t0 * v[a];
        double f = X[a] / G->d[a];
        int i = (int)floor(f);
        if (v[a] < 0.0 && f == floor(f)) i -= 1;
        if (i < 0) i = 0;
        if (i > G->n[a] - 1) i = G->n[a] - 1;
        vox[a] = i;
    }
    walker wk;
    walker_init(&wk, G, X, v, vox);
    double r = t1 - t0;
    int n = 0;
    for (;;) {
        int a = walker_axis(&wk);
        int last = wk.tmax[a] >= r;
        double tn = last ? r : wk.tmax[a];
        if (n < cap) {
            ks[n] = vox_index(G, wk.i);
            ls[n] = tn - wk.t;
            ++n;
        }
        if (last) break;
        if (walker_cross(&wk, G, a) != LEFT_NONE) break;
    }
    return n;
}

static void geom_of(const orc_grid* grid, geom* G)
{
    G->n[0] = grid->nx;
    G->n[1] = grid->ny;
    G->n[2] = grid->nz;
    G->d[0] = grid->dx;
    G->d[1] = grid->dy;
    G->d[2] = grid->dz;
}

/* Eq. (Jc) from a FMC run without local estimation: the tallies L_c(k) of
 * Eq. (Lcupdate), scaled by mu0 A_top / N, divided by beta(k). */
int oracle_voxel_scatter(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                         const orc_params* P, double* j, orc_stats* stats)
{
    int err = validate(grid, beta, n_cams, cams, P);
    if (err) return err;
    if (!j) return ORC_ERR_INVALID_ARG;
    int64_t nv = (int64_t)grid->nx * grid->ny * grid->nz;
    ctx c;
    ctx_setup(&c, grid, beta, beta, n_cams, cams, P, MODE_VOXEL);
    c.Lc = j;
    memset(j, 0, (size_t)n_cams * (size_t)nv * sizeof(double));
    run_photons(&c);
    uint64_t N = P->n_photons_norm ? P->n_photons_norm : P->n_photons;
    double base = N ? cos(P->sun_zenith) * c.L[0] * c.L[1] / (double)N : 0.0;
    for (int ci = 0; ci < n_cams; ++ci)
        for (int64_t k = 0; k < nv; ++k) {
            double* x = &j[(int64_t)ci * nv + k];
            *x = beta[k] > 0.0 ? *x * base / beta[k] : 0.0;
        }
    if (stats) *stats = c.st;
    ctx_free(&c);
    return ORC_OK;
}

static void voxel_centre(const geom* G, int64_t k, double X[3])
{
    int64_t nxy = (int64_t)G->n[0] * G->n[1];
    int ix = (int)(k % G->n[0]), iy = (int)((k / G->n[0]) % G->n[1]), iz = (int)(k / nxy);
    X[0] = (ix + 0.5) * G->d[0];
    X[1] = (iy + 0.5) * G->d[1];
    X[2] = (iz + 0.5) * G->d[2];
}

/* Eqs. (taoKtoc, Tck): T_c(k) = exp(-tau) along the LOS from the centre of
 * voxel k to camera c.  T: [camera][voxel]. */
int oracle_voxel_transmittance(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                               double* T)
{
    if (!grid || !beta || !cams || !T || n_cams < 1) return ORC_ERR_INVALID_ARG;
    geom G;
    geom_of(grid, &G);
    int64_t nv = (int64_t)grid->nx * grid->ny * grid->nz;
    for (int ci = 0; ci < n_cams; ++ci)
        for (int64_t k = 0; k < nv; ++k) {
            double X[3];
            voxel_centre(&G, k, X);
            T[(int64_t)ci * nv + k] = exp(-oracle_optical_depth(grid, beta, X, cams[ci].pos, NULL));
        }
    return ORC_OK;
}

/* Unit direction of sub-pixel ray (a, b) of pixel (row, col), n x n per
 * pixel (Eq. PIc): through the image point (col + (a + 1/2)/n,
 * row + (b + 1/2)/n), back-projected from the camera centre. */
static void subpixel_ray(const orc_camera* cam, int row, int col, int a, int b, int n, double v[3])
{
    double u = col + (a + 0.5) / n, w = row + (b + 0.5) / n;
    double q[3] = {(u - cam->cx) / cam->fx, (w - cam->cy) / cam->fy, 1.0};
    for (int i = 0; i < 3; ++i) v[i] = cam->R[i] * q[0] + cam->R[3 + i] * q[1] + cam->R[6 + i] * q[2];
    double len = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int i = 0; i < 3; ++i) v[i] /= len;
}

/* Eqs. (IcPJbetaT, Icpixel): i_c(p) = 1/(N_rays V) sum_rho sum_k
 * l_rho(k) j_c(k) beta(k) T_c(k), N_rays = n^2, no direct sunlight. */
int oracle_voxel_render(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                        int n, const double* j, double* images)
{
    if (!grid || !beta || !cams || !j || !images || n_cams < 1 || n < 1) return ORC_ERR_INVALID_ARG;
    geom G;
    geom_of(grid, &G);
    int64_t nv = (int64_t)grid->nx * grid->ny * grid->nz;
    double V = grid->dx * grid->dy * grid->dz;
    double* T = (double*)malloc((size_t)n_cams * (size_t)nv * sizeof(double));
    oracle_voxel_transmittance(grid, beta, n_cams, cams, T);
    int cap = grid->nx + grid->ny + grid->nz + 4;
    int64_t* ks = (int64_t*)malloc((size_t)cap * sizeof(int64_t));
    double* ls = (double*)malloc((size_t)cap * sizeof(double));
    int64_t off = 0;
    for (int ci = 0; ci < n_cams; ++ci) {
        const orc_camera* cam = &cams[ci];
        const double* jc = j + (int64_t)ci * nv;
        const double* Tc = T + (int64_t)ci * nv;
        for (int row = 0; row < cam->height; ++row)
            for (int col = 0; col < cam->width; ++col) {
                double acc = 0.0;
                for (int b = 0; b < n; ++b)
                    for (int a = 0; a < n; ++a) {
                        double v[3];
                        subpixel_ray(cam, row, col, a, b, n, v);
                        int m = segment_voxels(&G, cam->pos, v, INFINITY, ks, ls, cap);
                        for (int q = 0; q < m; ++q) acc += ls[q] * jc[ks[q]] * beta[ks[q]] * Tc[ks[q]];
                    }
                images[off + (int64_t)row * cam->width + col] = acc / ((double)n * n * V);
            }
        off += (int64_t)cam->width * cam->height;
    }
    free(ks);
    free(ls);
    free(T);
    return ORC_OK;
}

/* Gradient of L(i(beta)) for dL/di = dl with j frozen, Eqs. (Jaco1,
 * TcofJaco1, DivTc):  with B_c = Pi_c^T dl_c,
 * grad(m) = sum_c [ T_c(m) j_c(m) B_c(m)
 *                   - sum_k D_c(k, m) T_c(k) beta(k) j_c(k) B_c(k) ],
 * D_c(k, m) the length of the LOS from the centre of k to camera c in m.
 * With q (nullable, [camera][voxel]) camera c's term at voxel m is
 * multiplied by q_c(m): the conditioning Q_c of Eq. (divCost1). */
int oracle_voxel_grad(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                      int n, const double* j, const double* dl, const double* q, double* grad)
{
    if (!grid || !beta || !cams || !j || !dl || !grad || n_cams < 1 || n < 1) return ORC_ERR_INVALID_ARG;
    geom G;
    geom_of(grid, &G);
    int64_t nv = (int64_t)grid->nx * grid->ny * grid->nz;
    double V = grid->dx * grid->dy * grid->dz;
    double* T = (double*)malloc((size_t)n_cams * (size_t)nv * sizeof(double));
    double* B = (double*)calloc((size_t)nv, sizeof(double));
    oracle_voxel_transmittance(grid, beta, n_cams, cams, T);
    int cap = grid->nx + grid->ny + grid->nz + 4;
    int64_t* ks = (int64_t*)malloc((size_t)cap * sizeof(int64_t));
    double* ls = (double*)malloc((size_t)cap * sizeof(double));
    memset(grad, 0, (size_t)nv * sizeof(double));
    int64_t off = 0;
    for (int ci = 0; ci < n_cams; ++ci) {
        const orc_camera* cam = &cams[ci];
        const double* jc = j + (int64_t)ci * nv;
        const double* Tc = T + (int64_t)ci * nv;
        const double* qc = q ? q + (int64_t)ci * nv : NULL;
        /* B_c = Pi_c^T dl_c */
        memset(B, 0, (size_t)nv * sizeof(double));
        for (int row = 0; row < cam->height; ++row)
            for (int col = 0; col < cam->width; ++col) {
                double g = dl[off + (int64_t)row * cam->width + col];
                if (g == 0.0) continue;
                for (int b = 0; b < n; ++b)
                    for (int a = 0; a < n; ++a) {
                        double v[3];
                        subpixel_ray(cam, row, col, a, b, n, v);
                        int m = segment_voxels(&G, cam->pos, v, INFINITY, ks, ls, cap);
                        for (int q = 0; q < m; ++q) B[ks[q]] += g * ls[q] / ((double)n * n * V);
                    }
            }
        for (int64_t k = 0; k < nv; ++k) {
            if (B[k] == 0.0 || jc[k] == 0.0) continue;
            grad[k] += (qc ? qc[k] : 1.0) * Tc[k] * jc[k] * B[k];
            double w = Tc[k] * beta[k] * jc[k] * B[k];
            if (w == 0.0) continue;
            /* the LOS from the centre of k towards the camera */
            double X[3], D[3];
            voxel_centre(&G, k, X);
            for (int a = 0; a < 3; ++a) D[a] = cam->pos[a] - X[a];
            double len = sqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
            if (!(len > 0.0)) continue;
            for (int a = 0; a < 3; ++a) D[a] /= len;
            int m = segment_voxels(&G, X, D, len, ks, ls, cap);
            for (int t = 0; t < m; ++t) grad[ks[t]] -= (qc ? qc[ks[t]] : 1.0) * w * ls[t];
        }
        off += (int64_t)cam->width * cam->height;
    }
    free(ks);
    free(ls);
    free(B);
    free(T);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Recovery (Secs. 5.2, 6, 7): conditioning, regularisation, the surrogate  */
/* gradient-descent loop and the error measures.                            */

/* Sec. 6: Q_c(k, k) from the number of sub-pixel rays R_{c,p}^rho that pass
 * through voxel k (a length inside it above 1e-9 of the shortest voxel
 * edge, so that rounding does not decide whether a grazing ray counts).  counts: [camera][voxel].
 * The conditioned step divides by the count (q = 1/count, 0 where no ray
 * passes): a voxel seen by more rays gets a proportionally smaller step. */
int oracle_voxel_conditioning(const orc_grid* grid, int n_cams, const orc_camera* cams, int n,
                              double* counts, double* q)
{
    if (!grid || !cams || n_cams < 1 || n < 1) return ORC_ERR_INVALID_ARG;
    geom G;
    geom_of(grid, &G);
    int64_t nv = (int64_t)grid->nx * grid->ny * grid->nz;
    double* cnt = (double*)calloc((size_t)n_cams * (size_t)nv, sizeof(double));
    int cap = grid->nx + grid->ny + grid->nz + 4;
    int64_t* ks = (int64_t*)malloc((size_t)cap * sizeof(int64_t));
    double* ls = (double*)malloc((size_t)cap * sizeof(double));
    /* a ray that only grazes a voxel (an edge or corner) is not counted */
    double eps = 1e-9 * fmin(grid->dx, fmin(grid->dy, grid->dz));
    for (int ci = 0; ci < n_cams; ++ci) {
        const orc_camera* cam = &cams[ci];
        for (int row = 0; row < cam->height; ++row)
            for (int col = 0; col < cam->width; ++col)
                for (int b = 0; b < n; ++b)
                    for (int a = 0; a < n; ++a) {
                        double v[3];
                        subpixel_ray(cam, row, col, a, b, n, v);
                        int m = segment_voxels(&G, cam->pos, v, INFINITY, ks, ls, cap);
                        for (int t = 0; t < m; ++t)
                            if (ls[t] > eps) cnt[(int64_t)ci * nv + ks[t]] += 1.0;
                    }
    }
    for (int64_t i = 0; i < (int64_t)n_cams * nv; ++i) {
        if (counts) counts[i] = cnt[i];
        if (q) q[i] = cnt[i] > 0.0 ? 1.0 / cnt[i] : 0.0;
    }
    free(ks);
    free(ls);
    free(cnt);
    return ORC_OK;
}

/* Sec. 6: Psi(beta) = || W Lap beta ||^2 with Lap the 7-point Laplacian in
 * voxel units (a neighbour outside the domain takes the voxel's own value,
 * i.e. no flux through the boundary) and W diagonal, w_layer[iz] for the
 * voxels of layer iz (NULL: 1).  Returns Psi; grad (nullable) gets
 * 2 Lap^T W^T W Lap beta. */
static double lap_at(const geom* G, const double* f, int ix, int iy, int iz)
{
    int64_t k = (int64_t)ix + (int64_t)G->n[0] * ((int64_t)iy + (int64_t)G->n[1] * iz);
    double c = f[k], sum = -6.0 * c;
    int i[3] = {ix, iy, iz};
    for (int a = 0; a < 3; ++a)
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            int jn[3] = {i[0], i[1], i[2]};
            jn[a] += sgn;
            if (jn[a] < 0 || jn[a] >= G->n[a]) {
                sum += c;
            } else {
                sum += f[(int64_t)jn[0] + (int64_t)G->n[0] * ((int64_t)jn[1] + (int64_t)G->n[1] * jn[2])];
            }
        }
    return sum;
}

double oracle_laplacian_reg(const orc_grid* grid, const double* beta, const double* w_layer, double* grad)
{
    geom G;
    geom_of(grid, &G);
    int64_t nv = (int64_t)grid->nx * grid->ny * grid->nz;
    double* r = (double*)malloc((size_t)nv * sizeof(double));  /* W^2 Lap beta */
    double psi = 0.0;
    for (int iz = 0; iz < G.n[2]; ++iz)
        for (int iy = 0; iy < G.n[1]; ++iy)
            for (int ix = 0; ix < G.n[0]; ++ix) {
                double w = w_layer ? w_layer[iz] : 1.0;
                double l = lap_at(&G, beta, ix, iy, iz);
                psi += (w * l) * (w * l);
                r[(int64_t)ix + (int64_t)G.n[0] * ((int64_t)iy + (int64_t)G.n[1] * iz)] = w * w * l;
            }
    if (grad) {
        /* Lap is symmetric (each boundary term folds into the diagonal), so
         * Lap^T r = Lap r */
        for (int iz = 0; iz < G.n[2]; ++iz)
            for (int iy = 0; iy < G.n[1]; ++iy)
                for (int ix = 0; ix < G.n[0]; ++ix)
                    grad[(int64_t)ix + (int64_t)G.n[0] * ((int64_t)iy + (int64_t)G.n[1] * iz)] =
                        2.0 * lap_at(&G, r, ix, iy, iz);
    }
    free(r);
    return psi;
}

/* Eq. (noise): measured radiance to 10-bit grey levels.  scale = 2^10 over
 * the largest masked pixel of all cameras; out = the rounded (floor(x+1/2))
 * value of images * scale + 0.4 * normals, clipped to [0, 1024]. */
double oracle_camera_noise(int64_t n_pix, const double* images, const double* mask, const double* normals,
                           double* out)
{
    double mx = 0.0;
    for (int64_t p = 0; p < n_pix; ++p) {
        double v = (mask ? mask[p] : 1.0) * images[p];
        if (v > mx) mx = v;
    }
    double scale = mx > 0.0 ? 1024.0 / mx : 0.0;
    for (int64_t p = 0; p < n_pix; ++p) {
        double x = floor(images[p] * scale + 0.4 * normals[p] + 0.5);
        out[p] = x < 0.0 ? 0.0 : (x > 1024.0 ? 1024.0 : x);
    }
    return scale;
}

/* Sec. 7: delta_mass = (|b|_1 - |t|_1) / |t|_1, eps = |b - t|_1 / |t|_1. */
void oracle_recovery_error(int64_t n, const double* beta_hat, const double* beta_true, double out[2])
{
    double a = 0.0, t = 0.0, d = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        a += fabs(beta_hat[k]);
        t += fabs(beta_true[k]);
        d += fabs(beta_hat[k] - beta_true[k]);
    }
    out[0] = (a - t) / t;
    out[1] = d / t;
}

/* Sec. 5.2, Eqs. (Cost, divCost1, minobjectiveBetaQplus1, GD): n_outer
 * surrogate iterations.  Iteration q renders j at the current beta with the
 * photons of seed P->seed + q (Sec. 3.2), then takes n_gd gradient steps
 * of E(beta | j) = sum_c |M_c (i_c(beta | j) - measured_c)|^2
 *                  + eta Psi(beta),
 * beta <- max(beta - delta * grad, 0) (the non-negative set), grad =
 * 2 sum_c Q_c J_c^T M_c^2 (i_c - measured_c) + eta dPsi/dbeta, Q_c the
 * conditioning: 1 / count (conditioned = 1), the count of rays itself as the
 * passage words it (conditioned = 2), or 1 (0).  beta (in) is the start, (out) the
 * result; cost[q * n_gd + d] gets E before step d of iteration q. */
int oracle_recover(const orc_grid* grid, double* beta, int n_cams, const orc_camera* cams,
                   const orc_params* P, int n, const double* measured, const double* mask,
                   const double* w_layer, double eta, double delta, int n_gd, int n_outer, int conditioned,
                   double* cost)
{
    int err = validate(grid, beta, n_cams, cams, P);
    if (err) return err;
    if (!measured || n < 1 || n_gd < 1 || n_outer < 0) return ORC_ERR_INVALID_ARG;
    int64_t nv = (int64_t)grid->nx * grid->ny * grid->nz;
    int64_t npix = 0;
    for (int ci = 0; ci < n_cams; ++ci) npix += (int64_t)cams[ci].width * cams[ci].height;
    double* j = (double*)malloc((size_t)n_cams * (size_t)nv * sizeof(double));
    double* q = conditioned ? (double*)malloc((size_t)n_cams * (size_t)nv * sizeof(double)) : NULL;
    double* img = (double*)malloc((size_t)npix * sizeof(double));
    double* dl = (double*)malloc((size_t)npix * sizeof(double));
    double* g = (double*)malloc((size_t)nv * sizeof(double));
    double* gr = (double*)malloc((size_t)nv * sizeof(double));
    if (q) oracle_voxel_conditioning(grid, n_cams, cams, n, conditioned == 2 ? q : NULL, conditioned == 2 ? NULL : q);
    for (int it = 0; it < n_outer; ++it) {
        orc_params Pq = *P;
        Pq.seed = P->seed + (uint64_t)it;
        oracle_voxel_scatter(grid, beta, n_cams, cams, &Pq, j, NULL);
        for (int d = 0; d < n_gd; ++d) {
            oracle_voxel_render(grid, beta, n_cams, cams, n, j, img);
            double E = 0.0;
            for (int64_t p = 0; p < npix; ++p) {
                double m = mask ? mask[p] : 1.0;
                double r = m * (img[p] - measured[p]);
                E += r * r;
                dl[p] = 2.0 * m * r;
            }
            oracle_voxel_grad(grid, beta, n_cams, cams, n, j, dl, q, g);
            if (eta != 0.0) {
                E += eta * oracle_laplacian_reg(grid, beta, w_layer, gr);
                for (int64_t k = 0; k < nv; ++k) g[k] += eta * gr[k];
            }
            if (cost) cost[(int64_t)it * n_gd + d] = E;
            for (int64_t k = 0; k < nv; ++k) {
                double b = beta[k] - delta * g[k];
                beta[k] = b > 0.0 ? b : 0.0;
            }
        }
    }
    free(j);
    free(q);
    free(img);
    free(dl);
    free(g);
    free(gr);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Backward Monte Carlo (Sec. 2.1.4): per pixel, photon packets back-traced  */
/* from the camera, with the local estimate towards the sun, Eq. (ble).     */

/* Optical depth from X (in voxel vox) along unit v to the domain exit, and
 * the face it leaves through. */
static double tau_to_exit(ctx* c, const double X[3], const int vox[3], const double v[3], int* face)
{
    walker wk;
    walker_init(&wk, &c->G, X, v, vox);
    double tau = 0.0;
    for (;;) {
        int a = walker_axis(&wk);
        tau += c->beta_t[vox_index(&c->G, wk.i)] * (wk.tmax[a] - wk.t);
        int left = walker_cross(&wk, &c->G, a);
        if (left != LEFT_NONE) {
            *face = left;
            return tau;
        }
    }
}

/* Image of every camera by BMC with n_pp packets per pixel.  Packet i of
 * global pixel p has photon id p * n_pp + i: leg 0 gives the point of the
 * pixel (two uniforms) and the first free path; leg s >= 1 follows
 * collision s as in the forward method (polar, azimuth, roulette, free
 * path).  Steps: (i) start at the camera centre along the back-projected
 * direction through that point, entering the domain where the ray does;
 * (ii)-(iii) free flight, the packet ends when it leaves (a packet reaching
 * the sun directly has zero measure for a pinhole and is not counted);
 * at every collision the local estimate albedo I_s P(angle between the ray
 * and the direction to the sun) t(X -> sun), with t = 0 when the path to
 * the sun leaves through a side face (light enters through the top face
 * only, as in the forward method); (v) albedo and roulette, (vi) HG
 * scattering about the ray.  pixel = mean of the packets' sums: radiance
 * per unit solar irradiance, the units of the forward images; images_m2
 * (nullable) = mean of the squared packet sums. */
int oracle_bmc_render(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                      const orc_params* P, uint32_t n_pp, double* images, double* images_m2, orc_stats* stats)
{
    int err = validate(grid, beta, n_cams, cams, P);
    if (err) return err;
    if (!images || n_pp < 1) return ORC_ERR_INVALID_ARG;
    ctx c;
    ctx_setup(&c, grid, beta, beta, n_cams, cams, P, MODE_RENDER);
    double to_sun[3] = {-c.w_sun[0], -c.w_sun[1], -c.w_sun[2]};
    int64_t gp = 0;
    for (int ci = 0; ci < n_cams; ++ci) {
        const orc_camera* cam = &cams[ci];
        for (int row = 0; row < cam->height; ++row)
            for (int col = 0; col < cam->width; ++col, ++gp) {
                double sum = 0.0, sum2 = 0.0;
                for (uint32_t i = 0; i < n_pp; ++i) {
                    uint64_t pid = (uint64_t)gp * n_pp + i;
                    double packet = 0.0;
                    double u[4];
                    draw(P->seed, pid, 0u, u);
                    c.st.photons++;
                    /* (i) the ray through the point (col + u0, row + u1) */
                    double q[3] = {(col + u[0] - cam->cx) / cam->fx, (row + u[1] - cam->cy) / cam->fy, 1.0};
                    double d[3];
                    for (int a = 0; a < 3; ++a)
                        d[a] = cam->R[a] * q[0] + cam->R[3 + a] * q[1] + cam->R[6 + a] * q[2];
                    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                    for (int a = 0; a < 3; ++a) d[a] /= len;
                    double t0 = 0.0, t1 = INFINITY;
                    for (int a = 0; a < 3; ++a) {
                        if (d[a] == 0.0) {
                            if (cam->pos[a] < 0.0 || cam->pos[a] > c.L[a]) t1 = -1.0;
                            continue;
                        }
                        double ta = (0.0 - cam->pos[a]) / d[a], tb = (c.L[a] - cam->pos[a]) / d[a];
                        if (ta > tb) { double tmp = ta; ta = tb; tb = tmp; }
                        if (ta > t0) t0 = ta;
                        if (tb < t1) t1 = tb;
                    }
                    if (!(t1 > t0)) {
                        c.st.esc_side++;
                        continue;
                    }
                    double X[3];
                    int vox[3];
                    for (int a = 0; a < 3; ++a) {
                        X[a] = cam->pos[a] + t0 * d[a];
                        double f = X[a] / c.G.d[a];
                        int k = (int)floor(f);
                        if (d[a] < 0.0 && f == floor(f)) k -= 1;
                        if (k < 0) k = 0;
                        if (k > c.G.n[a] - 1) k = c.G.n[a] - 1;
                        vox[a] = k;
                    }
                    double weight = 1.0, tau_star = -log(1.0 - u[2]);
                    uint32_t s = 0;
                    for (;;) {
                        int left = free_flight(&c, X, vox, d, tau_star);
                        if (left != LEFT_NONE) {
                            if (left == ORC_FATE_TOP) c.st.esc_top++;
                            else if (left == ORC_FATE_BOTTOM) c.st.esc_bottom++;
                            else c.st.esc_side++;
                            break;
                        }
                        ++s;
                        c.st.events++;
                        /* Eq. (ble) */
                        int face = 0;
                        double tau = tau_to_exit(&c, X, vox, to_sun, &face);
                        c.st.le_jobs++;
                        if (face == ORC_FATE_TOP) {
                            double cosang = d[0] * to_sun[0] + d[1] * to_sun[1] + d[2] * to_sun[2];
                            packet += P->albedo * weight * oracle_hg_phase(P->g, cosang) * exp(-tau);
                        }
                        if (s >= P->max_events) {
                            c.st.capped++;
                            break;
                        }
                        draw(P->seed, pid, s, u);
                        weight *= P->albedo;
                        if (weight < P->rr_weight) {
                            if (u[2] < weight / P->rr_weight) {
                                weight = P->rr_weight;
                            } else {
                                c.st.rr_killed++;
                                break;
                            }
                        }
                        double mu = oracle_hg_sample(P->g, u[0]);
                        double wn[3];
                        oracle_scatter_direction(d, mu, 2.0 * ORC_PI * u[1], wn);
                        d[0] = wn[0];
                        d[1] = wn[1];
                        d[2] = wn[2];
                        tau_star = -log(1.0 - u[3]);
                    }
                    sum += packet;
                    sum2 += packet * packet;
                }
                images[gp] = sum / (double)n_pp;
                if (images_m2) images_m2[gp] = sum2 / (double)n_pp;
            }
    }
    if (stats) *stats = c.st;
    ctx_free(&c);
    return ORC_OK;
}
