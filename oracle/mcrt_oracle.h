/*
 * CPU oracle for forward Monte Carlo with local estimation to in-situ
 * cameras, and for the surrogate (frozen in-scatter) gradient of an image
 * loss with respect to the extinction grid.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64
 * implementation written from the paper (Holodovsky et al., "In-situ
 * multi-scattering tomography", arXiv 1512.02110): the photon life cycle of
 * Sec. 2.1.2 (steps i-vi), the free path of Eqs. (Ftau, taurand, MCextinct),
 * the Henyey-Greenstein phase function Eq. (Phg) and its sampling
 * Eq. (thetaHG, squared form), the local estimate Eq. (fle) with the
 * transmittance Eqs. (beer-lambert, tc), and the surrogate Jacobian
 * Eqs. (Jaco1, TcofJaco1, DivTc) carried to one scattering event.  Only the
 * test-suite, the package's smoke check and the benchmark's CPU-baseline leg
 * may load it; the GPU library never does.  It shares no code with the GPU
 * library.
 *
 * All arrays are host memory owned by the caller.  Functions return 0 on
 * success and a negative ORC_ERR_* code on invalid input.
 */
#ifndef MCRT_ORACLE_H
#define MCRT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_ERR_INVALID_ARG = -1 };

/* Voxel grid, Sec. 3: domain [0,nx dx] x [0,ny dy] x [0,nz dz] km, z up,
 * voxel k = ix + nx*(iy + ny*iz). */
typedef struct {
    int32_t nx, ny, nz, pad_;
    double dx, dy, dz;
} orc_grid;

/* Pinhole camera: q = R (X - pos), column u = fx qx/qz + cx, row v = fy qy/qz + cy,
 * image [height][width], pixel (row, col) = (floor v, floor u). */
typedef struct {
    double pos[3];
    double R[9];
    double fx, fy, cx, cy;
    int32_t width, height;
} orc_camera;

typedef struct {
    double albedo;        /* single-scattering albedo, [0,1] */
    double g;             /* HG asymmetry, (-1,1) */
    double sun_zenith;    /* rad, [0, pi/2): zenith of the direction towards the sun */
    double sun_azimuth;   /* rad, from +x towards +y */
    double rr_weight;     /* Russian-roulette threshold weight, (0,1] */
    uint64_t n_photons;   /* photons traced: ids photon_offset .. photon_offset+n_photons-1 */
    uint64_t seed;
    uint64_t photon_offset;
    uint64_t n_photons_norm; /* photon count used in the image normalisation; 0 = n_photons */
    uint32_t max_events;  /* collisions per photon before it is stopped (>=1) */
    int32_t pad_;
} orc_params;

typedef struct {
    uint64_t photons, events, le_jobs, vox_free, vox_conn;
    uint64_t esc_top, esc_bottom, esc_side, rr_killed, capped;
} orc_stats;

/* One scattering event of a traced path. */
typedef struct {
    double x, y, z;       /* collision point */
    double w;             /* packet weight I_s at the event (before albedo) */
    int32_t voxel;        /* voxel of the collision */
    int32_t pad_;
} orc_event;

enum { ORC_FATE_TOP = 0, ORC_FATE_BOTTOM = 1, ORC_FATE_SIDE = 2, ORC_FATE_RR = 3, ORC_FATE_CAP = 4 };

typedef struct {
    int32_t n_events;     /* collisions of the photon (may exceed max_rec) */
    int32_t fate;         /* ORC_FATE_* */
    double exit_pos[3];   /* where the photon left the domain (fates TOP/BOTTOM/SIDE) */
    double exit_dir[3];   /* its direction there */
    double exit_w;        /* and its weight */
} orc_path;

/* Forward render.  images: sum over cameras of height*width doubles,
 * [cam][row][col], overwritten with radiance per unit solar irradiance.
 * images_m2 (nullable): per pixel, the sum over photons of the square of
 * each photon's normalised contribution (for Monte Carlo error bars).
 * stats (nullable). */
int oracle_render(const orc_grid* grid, const double* beta, int n_cams,
                  const orc_camera* cams, const orc_params* prm,
                  double* images, double* images_m2, orc_stats* stats);

/* Frozen-event render: photons are transported through beta_sample; each
 * local estimate is evaluated with beta_eval, i.e. scaled by
 * beta_eval(k_e)/beta_sample(k_e) and attenuated by exp(-tau) of beta_eval.
 * With beta_eval == beta_sample this is oracle_render. */
int oracle_render_frozen(const orc_grid* grid, const double* beta_sample,
                         const double* beta_eval, int n_cams,
                         const orc_camera* cams, const orc_params* prm,
                         double* images, orc_stats* stats);

/* Surrogate gradient d L / d beta for given dL/d images (same layout as the
 * images), evaluated on the events of the forward render with the same
 * parameters.  grad: nx*ny*nz doubles, overwritten. */
int oracle_grad_beta(const orc_grid* grid, const double* beta, int n_cams,
                     const orc_camera* cams, const orc_params* prm,
                     const double* dl_dimages, double* grad, orc_stats* stats);

/* Per-photon event records for photon ids first_pid .. first_pid+count-1.
 * events: count*max_rec records; pix (nullable): count*max_rec*n_cams pixel
 * indices (row*width+col, or -1 when the camera does not see the event). */
int oracle_trace_paths(const orc_grid* grid, const double* beta, int n_cams,
                       const orc_camera* cams, const orc_params* prm,
                       uint64_t first_pid, uint32_t count, uint32_t max_rec,
                       orc_event* events, int32_t* pix, orc_path* paths);

/* ---- building blocks exposed for the pin tests ---- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double oracle_uniform(uint32_t x);
double oracle_hg_phase(double g, double cos_angle);
double oracle_hg_sample(double g, double u);
void oracle_scatter_direction(const double w_in[3], double mu, double phi, double w_out[3]);
/* Optical depth of the segment p0 -> p1 (parts outside the domain count 0);
 * nvox (nullable) receives the number of voxels visited. */
double oracle_optical_depth(const orc_grid* grid, const double* beta,
                            const double p0[3], const double p1[3], int64_t* nvox);
double oracle_pixel_solid_angle(const orc_camera* cam, int row, int col);

/* Voxelised forward model (Sec. 3).  Arrays [camera][voxel] hold one value
 * per camera and voxel (voxel index fastest).
 * oracle_voxel_scatter: FMC without local estimation; j = j_c(k) of Eq. (Jc)
 *   (L_c of Eq. (Lcupdate) times mu0 A_top / N, over beta; 0 where beta = 0).
 * oracle_voxel_transmittance: T = T_c(k) of Eq. (Tck), LOS from the voxel
 *   centre to the camera centre.
 * oracle_voxel_render: i_c(p) of Eq. (Icpixel) with n x n sub-pixel rays.
 * oracle_voxel_grad: dL/dbeta for image gradient dl with j frozen, Eqs.
 *   (Jaco1, TcofJaco1, DivTc). */
int oracle_voxel_scatter(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                         const orc_params* prm, double* j, orc_stats* stats);
int oracle_voxel_transmittance(const orc_grid* grid, const double* beta, int n_cams,
                               const orc_camera* cams, double* T);
int oracle_voxel_render(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                        int n, const double* j, double* images);
int oracle_voxel_grad(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                      int n, const double* j, const double* dl, const double* q, double* grad);

/* Recovery (Secs. 5.2, 6, 7).
 * oracle_voxel_conditioning: counts[c][k] = sub-pixel rays of camera c that
 *   cross voxel k; q = 1/counts (0 where none); either output nullable.
 * oracle_laplacian_reg: Psi = |W Lap beta|^2 (7-point Laplacian in voxel
 *   units, no flux through the boundary, W = w_layer[iz] or 1); grad
 *   (nullable) = 2 Lap^T W^2 Lap beta.
 * oracle_camera_noise: Eq. (noise) with the caller's N(0,1) draws; returns
 *   the grey-level scale.
 * oracle_recovery_error: out = {delta_mass, eps} of Sec. 7.
 * oracle_recover: the surrogate gradient-descent loop (see the source);
 *   conditioned: 0 none, 1 Q_c = 1/counts, 2 Q_c = counts. */
/* Backward Monte Carlo (Sec. 2.1.4, Eq. ble): n_pp packets per pixel;
 * images in the units of oracle_render's (see the source for the steps and
 * the photon ids).  prm->n_photons and photon_offset are not used. */
int oracle_bmc_render(const orc_grid* grid, const double* beta, int n_cams, const orc_camera* cams,
                      const orc_params* prm, uint32_t n_pp, double* images, double* images_m2,
                      orc_stats* stats);

/* Air + aerosol mixture (step iv; Eqs. Pray, thetaREY, channelBeta).  The
 * channel's extinction is beta_air + sigma * beta_aer (beta_aer: aerosol
 * field of the reference channel, sigma > 0 the ratio of the channel's
 * aerosol cross-section to the reference one); prm->albedo and prm->g are
 * the aerosol's, air scatters with albedo 1 and the Rayleigh phase function.
 * At each collision the particle is air with probability beta_air / beta in
 * the voxel (first word of Philox counter (pid_lo, pid_hi, s, 1)); the local
 * estimate and the scattering use that particle.  With beta_air = 0 this is
 * oracle_render on sigma * beta_aer.
 * oracle_grad_mix ADDS dL/d beta_aer (reference field) to grad: the
 * surrogate with the in-scatter field frozen (full = 0) or the full
 * derivative of the expected images, path probabilities included (full = 1);
 * see the source. */
int oracle_render_mix(const orc_grid* grid, const double* beta_air, const double* beta_aer, double sigma,
                      int n_cams, const orc_camera* cams, const orc_params* prm, double* images,
                      double* images_m2, orc_stats* stats);
int oracle_grad_mix(const orc_grid* grid, const double* beta_air, const double* beta_aer, double sigma,
                    int n_cams, const orc_camera* cams, const orc_params* prm, const double* dl_dimages,
                    int full, double* grad, orc_stats* stats);
double oracle_rayleigh_phase(double cos_angle);
double oracle_rayleigh_sample(double u);

int oracle_voxel_conditioning(const orc_grid* grid, int n_cams, const orc_camera* cams, int n,
                              double* counts, double* q);
double oracle_laplacian_reg(const orc_grid* grid, const double* beta, const double* w_layer, double* grad);
double oracle_camera_noise(int64_t n_pix, const double* images, const double* mask, const double* normals,
                           double* out);
void oracle_recovery_error(int64_t n, const double* beta_hat, const double* beta_true, double out[2]);
int oracle_recover(const orc_grid* grid, double* beta, int n_cams, const orc_camera* cams,
                   const orc_params* prm, int n, const double* measured, const double* mask,
                   const double* w_layer, double eta, double delta, int n_gd, int n_outer, int conditioned,
                   double* cost);

#ifdef __cplusplus
}
#endif
#endif
