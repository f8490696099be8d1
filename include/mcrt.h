/*
 * mcrt.h - C ABI of the MI355X (gfx950) Monte Carlo renderer for in-situ
 * multi-scattering tomography.
 *
 * Method: Holodovsky, Schechner, Levin, Levis, Aides, "In-situ
 * multi-scattering tomography", arXiv 1512.02110.
 *   - Forward Monte Carlo (FMC), Sec. 2.1.2 steps (i)-(vi): photons enter at
 *     the top of the domain along the sun direction, fly free paths drawn by
 *     inverse transform (Eqs. Ftau, taurand, MCextinct) through a voxel grid
 *     of piecewise-constant extinction (Sec. 3), lose albedo at every
 *     collision with Russian roulette below a weight threshold, and scatter
 *     with the Henyey-Greenstein phase function (Eqs. Phg, thetaHG).
 *   - Local estimation (Sec. 2.1.3, Eq. fle): at every collision, every
 *     camera that sees the collision point receives
 *     albedo * I_s * P(angle) * exp(-tau(X_s -> X_c)) / |X_c - X_s|^2 in the
 *     pixel hit by the connecting ray; tau is the optical depth of that ray
 *     (Eqs. tau, beer-lambert, tc).
 *   - Surrogate gradient (Sec. 5.2, Eqs. Jaco1, TcofJaco1, DivTc): with the
 *     in-scatter field frozen at the events of the render, a local estimate
 *     C_e from a collision in voxel k_e has
 *     dC_e/dbeta(m) = C_e (delta(m, k_e) / beta(k_e) - l_e(m)),
 *     l_e(m) the length of the connecting ray inside voxel m.
 *
 * Conventions for every entry point:
 *   - Structs (grid, cameras, params, stats) are HOST memory and are read (or
 *     written, for stats) before the call returns.
 *   - Array arguments (beta, images, dl_dimages, grad_beta, trace buffers)
 *     are DEVICE pointers on the current HIP device, owned by the caller.
 *     The library never frees or keeps them.
 *   - Work is enqueued on `hip_stream` (a hipStream_t; NULL = the legacy
 *     default stream).  The call returns without waiting unless `stats` is
 *     non-NULL, in which case it waits for the stream and fills *stats.
 *   - The library allocates its own scratch (counters, the camera table,
 *     per-pixel weights and, for mc_grad_beta on large grids, the ray tape
 *     bounded by params->tape_limit) stream-ordered on `hip_stream` and
 *     releases it stream-ordered before returning.  The allocations come
 *     from a memory pool of the library (one per device) that keeps freed
 *     memory for later calls instead of returning it to the device, and the
 *     two large buffers (a kept render's rays, a gradient's bins) stay
 *     allocated between calls for reuse; mc_release_memory returns both.
 *   - 1 <= n_cams <= 65535; the pixels of all cameras number < 2^31.
 *   - Return value: MC_OK (0) or a negative MC_ERR_* code; the library never
 *     prints or aborts.  On an argument error nothing is enqueued.  On
 *     MC_ERR_HIP the contents of output arrays are unspecified.
 *   - beta must be finite and >= 0 (a negative or NaN value yields
 *     meaningless images but every kernel still terminates).
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = seed
 *     and counter (photon id lo, photon id hi, leg, 0); leg 0 launches the
 *     photon (uniforms: x, y, free path), leg s >= 1 follows collision s
 *     (uniforms: polar, azimuth, roulette, free path).  A uniform is
 *     ((word >> 9) + 1/2) * 2^-23.  The same (seed, photon id) gives the same
 *     photon on every run, device and precision, up to rounding.
 *   - Environment: MC_PLAIN_WALK_LOADS=1 (read at every call) makes the
 *     connection walks read beta with plain loads, the path that grids too
 *     large for the walks' buffer (n_vox times the walk's element size of
 *     2^31 bytes or more) always take; results are the same up to the order
 *     of the FP64 atomic sums.  Meant for testing that path on small grids.
 */
#ifndef MCRT_H
#define MCRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MC_OK = 0,
    MC_ERR_INVALID_ARG = -1,   /* an argument is out of range or a pointer is missing */
    MC_ERR_NO_DEVICE = -2,     /* no HIP device is visible */
    MC_ERR_HIP = -3,           /* a HIP runtime call or kernel launch failed */
    MC_ERR_OUT_OF_MEMORY = -4, /* scratch allocation failed */
    MC_ERR_SCRATCH_LIMIT = -5  /* mc_render_noalloc: the call needs more than its fixed scratch */
};

/* Transport precision.  Connection-ray optical depths and all tallies are
 * FP64 in every mode, and so is the projection of a collision onto a camera
 * (its pixel and the cull at the camera centre).
 *   MC_FP32: photon state (position, direction, weight), free flights,
 *     scattering and the connection-ray walks in FP32; beta is float.
 *   MC_FP64: all of it in FP64; beta is double.
 *   MC_MIXED: the photons (launch, free flights, collisions, roulette,
 *     scattering) in FP64, exactly as MC_FP64, and the walks of the
 *     connection rays -- most of the voxel steps -- in FP32 over a float copy
 *     of beta; beta is double.  The photon paths, events, counters and pixels
 *     are those of MC_FP64; only the local estimates differ, by FP32
 *     rounding of the connection rays' optical depths (segment lengths and
 *     the float copy of beta) and of their transmittance exp(-tau).
 *     Accepted by mc_render, mc_render_moments, mc_render_noalloc,
 *     mc_render_tape (which then keeps no tape), mc_grad_beta (the gradient
 *     of the same events, computed with the FP64 walks) and mc_trace_paths
 *     (the FP64 paths); the other entry points return MC_ERR_INVALID_ARG. */
enum { MC_FP32 = 0, MC_FP64 = 1, MC_MIXED = 2 };

/* Tally accumulation: FP64 atomics, or FP32 sum + FP32 compensation term
 * (error-free transformation of every atomic add), reduced to FP64 at the
 * end. */
enum { MC_TALLY_F64 = 0, MC_TALLY_KAHAN32 = 1 };

/* Voxel grid (Sec. 3): domain [0, nx*dx] x [0, ny*dy] x [0, nz*dz] in km, z up.
 * Voxel k = ix + nx*(iy + ny*iz) (x fastest), beta(k) in km^-1, constant
 * inside the voxel.  1 <= nx, ny <= 2048, 1 <= nz <= 1024, nx*ny*nz < 2^31,
 * d* > 0. */
typedef struct mc_grid {
    int32_t nx, ny, nz, pad_;
    double dx, dy, dz;
} mc_grid;

/* Pinhole camera c (Sec. 2.1, "center of projection X_c"; the cone of pixel
 * p is the set of directions that project into it).  A point X maps to
 * q = R (X - pos) (R row-major, rows = camera x-right, y-down, z-forward),
 * column u = fx qx/qz + cx and row v = fy qy/qz + cy; it is seen when qz > 0
 * and 0 <= u < width, 0 <= v < height, in pixel (floor v, floor u).
 * fx, fy > 0; width, height >= 1. */
typedef struct mc_camera {
    double pos[3];
    double R[9];
    double fx, fy, cx, cy;
    int32_t width, height;
} mc_camera;

typedef struct mc_params {
    double albedo;            /* single-scattering albedo, 0 <= albedo <= 1 */
    double g;                 /* HG asymmetry, -1 < g < 1 */
    double sun_zenith;        /* rad, 0 <= . < pi/2: zenith of the direction TO the sun */
    double sun_azimuth;       /* rad, from +x towards +y; photons travel along -s */
    double rr_weight;         /* Russian-roulette threshold weight, 0 < . <= 1 (0.1 typical) */
    uint64_t n_photons;       /* photons traced: ids photon_offset .. photon_offset + n_photons - 1 */
    uint64_t seed;            /* Philox key */
    uint64_t photon_offset;   /* first photon id */
    uint64_t n_photons_norm;  /* N in the image normalisation; 0 means n_photons.  Set it to
                                 the total of all shards when photon ranges are split. */
    uint32_t max_events;      /* collisions after which a photon is stopped and counted as
                                 capped, >= 1 */
    int32_t transport;        /* MC_FP32, MC_FP64 or MC_MIXED */
    int32_t tally;            /* MC_TALLY_F64 or MC_TALLY_KAHAN32 */
    int32_t tape_limit;       /* mc_grad_beta on grids too large for an LDS copy of the
                                 gradient: most records of its ray tape (stream-ordered
                                 scratch of 4 + 8 sizeof(real) bytes each); 0 = automatic
                                 (up to a quarter of free device memory, at most 32 GiB).
                                 A smaller tape means more, smaller replay chunks.  >= 0. */
} mc_params;

/* Counters of one call (all photons of the call). */
typedef struct mc_stats {
    uint64_t photons;     /* photons traced */
    uint64_t events;      /* collisions (scattering events), including a capped one */
    uint64_t le_jobs;     /* local estimates made (camera sees the collision) */
    uint64_t vox_free;    /* voxels visited by free flights */
    uint64_t vox_conn;    /* voxels visited by connection rays (one walk per local estimate) */
    uint64_t esc_top, esc_bottom, esc_side;  /* photons that left through each face */
    uint64_t rr_killed;   /* photons ended by Russian roulette */
    uint64_t capped;      /* photons stopped at max_events */
    double transport_ms;  /* device time of the transport kernel (all its launches), from
                             HIP events recorded on hip_stream around each launch */
    double tape_ms;       /* mc_grad_beta on large grids: device time of the binning and
                             deposit passes (events around each chunk's passes); else 0 */
} mc_stats;

/* Forward render (FMC + local estimation).
 * beta: device array of nx*ny*nz values, float for MC_FP32 transport and
 *   double for MC_FP64 and MC_MIXED.
 * images: device array of sum_c width_c*height_c doubles, [camera][row][col],
 *   overwritten with radiance per unit solar irradiance: the sum of local
 *   estimates of a pixel times mu0 * A_top / (N * Omega_p), with
 *   mu0 = cos(sun_zenith), A_top = nx dx ny dy, N = n_photons_norm (or
 *   n_photons) and Omega_p the solid angle of the pixel.  n_photons = 0
 *   yields zero images.
 * tally must be MC_TALLY_F64 or MC_TALLY_KAHAN32.
 * stats: nullable; non-NULL makes the call wait for the stream. */
int mc_render(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
              const mc_params* params, double* images, mc_stats* stats, void* hip_stream);

/* mc_render plus Monte Carlo error bars.  images_m2 (device, same layout as
 * images, nullable) is overwritten with the sum over local estimates of the
 * square of each normalised estimate; Var(image) ~= images_m2 - images^2 / N
 * (exact when no photon adds more than one estimate to a pixel, otherwise a
 * lower bound).  Costs one more FP64 atomic per local estimate. */
int mc_render_moments(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
                      const mc_params* params, double* images, double* images_m2, mc_stats* stats,
                      void* hip_stream);

/* mc_render without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid it).  Same arguments, images and counters as mc_render; the
 * library's scratch (counters, camera table, the copy of beta, the occupancy
 * bitmask, the compensated tally) lives in a fixed device array of 64 MiB
 * that every device the library runs on holds until the process ends.  The
 * call allocates nothing (no hipMalloc, no pool, no events): stats, when
 * non-NULL, report the counters with transport_ms = 0 and make the call wait
 * for the stream.  The scratch a call needs is about sizeof(real) bytes per
 * voxel (4 for MC_FP32 transport, 8 for MC_FP64), 8 bytes per pixel with
 * MC_TALLY_KAHAN32, and under 40 KB besides; a call that needs more than
 * 64 MiB (e.g. FP64 transport on 256 x 256 x 128 voxels) returns
 * MC_ERR_SCRATCH_LIMIT and enqueues nothing.  Every call on one device shares
 * that device's array and leaves its contents behind; calls that overlap on
 * one device (other streams, other threads) race and give wrong images:
 * serialise them. */
int mc_render_noalloc(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
                      const mc_params* params, double* images, mc_stats* stats, void* hip_stream);

/* Surrogate gradient dL/dbeta for a loss L(images) whose image gradient is
 * dl_dimages (device, same layout as mc_render's images; for an L2 loss,
 * 2 (i - i_measured) times any pixel mask).  The events are those of
 * mc_render with the same grid, beta, cameras and params (same seed and
 * photon range).
 * grad_beta: device array of nx*ny*nz doubles, overwritten.
 * Grids of more than about 7000 voxels (an FP64 gradient too large for a
 * per-workgroup LDS copy) are cut into tiles of at most 16384 voxels: the
 * photons are replayed in chunks whose connection rays are written to a
 * tape, once per tile crossed, then accumulated tile by tile in LDS.  Such
 * a call waits for the stream after every chunk (it reads back the tape's
 * fill to size the next chunk), whether or not stats is NULL. */
int mc_grad_beta(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
                 const mc_params* params, const double* dl_dimages, double* grad_beta,
                 mc_stats* stats, void* hip_stream);

/* Reverse mode with a stored tape instead of a replay.
 * mc_render_tape is mc_render that also keeps, in device memory the library
 * allocates, every connection ray of the render (start point, pixel, local
 * estimate C_e) for mc_grad_beta_tape, which then bins and deposits those
 * rays (Eq. DivTc with the weights of Sec. 5.2) without tracing the photons
 * again.  *tape is set to NULL (and the call still renders) when the grid
 * is small enough for mc_grad_beta's in-LDS gradient (no tape needed), when
 * the rays do not fit (params->tape_limit records if > 0, else three
 * eighths of the free device memory) or when the grid has too many tiles.
 * mc_render_tape always waits for the stream.
 * mc_grad_beta_tape: same contract as mc_grad_beta for the render that made
 * the tape: grid, cameras and every parameter except tally and tape_limit
 * must equal those of mc_render_tape (MC_ERR_INVALID_ARG otherwise), and
 * beta must hold the same values (not checked).  The tape is not consumed;
 * params->tape_limit bounds the bin space.  stats reports the render's
 * counters, transport_ms = 0 and the binning and deposit time in tape_ms.
 * mc_tape_free releases the tape's memory (stream-ordered on hip_stream, so
 * work already enqueued that reads it completes first); NULL is accepted.
 * A tape belongs to the device that was current for mc_render_tape. */
typedef struct mc_tape mc_tape;

int mc_render_tape(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
                   const mc_params* params, double* images, mc_stats* stats, void* hip_stream, mc_tape** tape);

int mc_grad_beta_tape(const mc_tape* tape, const mc_grid* grid, const void* beta, int n_cams,
                      const mc_camera* cams, const mc_params* params, const double* dl_dimages, double* grad_beta,
                      mc_stats* stats, void* hip_stream);

int mc_tape_free(mc_tape* tape, void* hip_stream);

/* Returns the device memory the library keeps for reuse on the current
 * device (its pool and its cached large buffers, except what a live tape or
 * a call in flight uses) to the device.  Call it when the streams the
 * library used are idle. */
int mc_release_memory(void);

/* Backward Monte Carlo (Sec. 2.1.4, Eq. ble): n_per_pixel packets per
 * pixel traced from the camera centre through a uniform point of the pixel,
 * with the forward method's free flights, albedo, roulette, HG scattering
 * and max_events; at every collision the local estimate
 * albedo I_s P(angle between the ray and the direction to the sun)
 * exp(-tau to the top face) (0 when the path to the sun leaves through a
 * side face: light enters through the top face only, as in mc_render).
 * Packet i of global pixel p has photon id p n_per_pixel + i: Philox leg 0
 * gives the point of the pixel (first two uniforms) and the first free path
 * (third); legs s >= 1 as in mc_render.  params->n_photons and
 * photon_offset are not used.  images (same layout and units as mc_render's)
 * = mean over the pixel's packets of their sums; images_m2 (nullable) = mean
 * of the squared sums (Var(image) = (images_m2 - images^2) / n_per_pixel).
 * tally must be MC_TALLY_F64; stats.photons = packets, le_jobs = events. */
int mc_bmc_render(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
                  const mc_params* params, uint32_t n_per_pixel, double* images, double* images_m2,
                  mc_stats* stats, void* hip_stream);

/* Frozen-event render (a test and diagnostic export): the photons are
 * transported through beta_sample, and every local estimate walks its
 * connection ray through beta_eval and is scaled by
 * beta_eval(k_e) / beta_sample(k_e) at its collision voxel k_e.  At
 * beta_eval = beta_sample this is mc_render; its derivative with respect to
 * beta_eval there is the surrogate gradient of mc_grad_beta (Sec. 5.2 with
 * the in-scatter field frozen, carried to one scattering event).  Both
 * fields in the transport precision (params->transport), device memory;
 * images and stats as in mc_render. */
int mc_render_frozen(const mc_grid* grid, const void* beta_sample, const void* beta_eval, int n_cams,
                     const mc_camera* cams, const mc_params* params, double* images, mc_stats* stats,
                     void* hip_stream);

/* Air + aerosol mixture, one colour channel (Sec. 2.1.2 step iv; Eqs.
 * (Pray), (thetaREY), (channelBeta)).  The channel's extinction is
 * beta = beta_air + sigma * beta_aer: beta_air (the known air field of the
 * channel) and beta_aer (the aerosol field of the reference channel) are
 * device FP64 arrays of nx*ny*nz values, x fastest, >= 0 (not checked);
 * sigma > 0 is the ratio of the channel's aerosol cross-section to the
 * reference one.  params->albedo and params->g describe the aerosol; air
 * scatters with albedo 1 and the Rayleigh phase function.  At collision s
 * of photon pid the particle is air when the first uniform of Philox
 * counter (pid_lo, pid_hi, s, 1) is below beta_air / beta in the collision
 * voxel (compared in FP64 for either transport precision); the local
 * estimate (albedo and phase function), the weight update and the sampled
 * scattering angle (Eq. thetaHG or thetaREY) are those of that particle.
 * With beta_air = 0 this is mc_render on sigma * beta_aer.  images,
 * images_m2 (nullable), stats as in mc_render_moments.  An RGB image is three
 * calls, one per channel (its beta_air and sigma). */
int mc_render_mixture(const mc_grid* grid, const double* beta_air, const double* beta_aer, double sigma,
                      int n_cams, const mc_camera* cams, const mc_params* params, double* images, double* images_m2,
                      mc_stats* stats, void* hip_stream);

/* Gradient of a loss with respect to the reference aerosol field beta_aer
 * for the render mc_render_mixture makes with the same arguments,
 * given dL/d images (device FP64, the images' layout), ADDED to
 * grad_beta_aer (device FP64, nx*ny*nz; zero it first; summing the calls of
 * the three channels gives the RGB gradient of Eq. (divCost1) for the
 * image term).  With a_e = dL/di(p) * mu0 A_top / (N Omega_p) * C_e for the
 * local estimate C_e of collision e (voxel k_e, particle t_e) and its
 * connection lengths l_e(m):
 *  full = 0: the surrogate with the in-scatter field frozen (Sec. 5.2):
 *      sigma * sum_e a_e ([t_e aerosol] delta(m,k_e) / beta_aer,ch(k_e) - l_e(m));
 *  full = 1: the derivative of the expected images, the probability of
 *      every photon path differentiated too: per photon, with free-flight
 *      lengths l_s(m) of the leg ending at collision s and A_s the sum of a
 *      over its collisions s and later,
 *      sigma * [sum_s A_s ([t_s aerosol] delta(m,k_s) / beta_aer,ch(k_s) - l_s(m))
 *               - sum_e a_e l_e(m)],
 *      by replaying each photon twice (once for the sum of its a).
 * (beta_aer,ch = sigma * beta_aer.)  When the grid's tiles fit the tile
 * bins, the photons are replayed with the forward's local-estimate queue and
 * every connection term becomes a ray record, binned by tile and deposited
 * in LDS (chunks of photons whose records fit params->tape_limit when > 0,
 * else the free memory); the full gradient's path terms follow each chunk,
 * one photon per lane with FP64 device atomics, reading the per-collision
 * sums of a that the replay kept (15 collisions per photon, the later ones
 * walked again).  Otherwise, or when params->tape_limit is too small for one
 * block of records, one photon per lane does everything, with records where
 * they fit and FP64 device atomics for the rest.  params->tally is ignored.
 * The result depends on the route only through FP64 summation order.
 * stats count the photons' first replay. */
int mc_grad_mixture(const mc_grid* grid, const double* beta_air, const double* beta_aer, double sigma, int n_cams,
                    const mc_camera* cams, const mc_params* params, const double* dl_dimages, int full,
                    double* grad_beta_aer, mc_stats* stats, void* hip_stream);

/* Voxelised forward model (Sec. 3) and its frozen-j gradient (Sec. 5.2).
 * Arrays "[camera][voxel]" are device arrays of n_cams * nx*ny*nz doubles,
 * camera-major, voxel index fastest.
 *
 * mc_voxel_scatter: forward Monte Carlo without local estimation (the same
 *   photons as mc_render for the same params); every collision in voxel k
 *   adds albedo I_s P(angle) to L_c(k) of every camera c, the angle between
 *   the incoming direction and the direction from the collision point to
 *   the camera centre (Eq. Lcupdate).  j is overwritten with
 *   j_c(k) = L_c(k) mu0 A_top / (N beta(k)) (Eq. Jc; 0 where beta(k) = 0),
 *   the in-scatter field in the units of the images.  beta is float for
 *   MC_FP32 transport, double for MC_FP64; tally must be MC_TALLY_F64.
 *   stats: le_jobs counts the (collision, camera) tallies.
 * mc_voxel_render: images (same layout as mc_render's) =
 *   i_c(p) = 1/(n^2 V) sum_rho sum_k l_rho(k) j_c(k) beta(k) T_c(k)
 *   (Eqs. IcP, PIc, Icpixel), n = rays_per_side: the rays from the camera
 *   centre through the n x n cell centres of the pixel; T_c(k) =
 *   exp(-tau) along the line of sight from the centre of voxel k to the
 *   camera centre (Eqs. taoKtoc, Tck); parts outside the domain contribute
 *   nothing; no direct sunlight.  beta is double.  Deterministic (FP64).
 * mc_voxel_grad: grad_beta = d/dbeta of sum_p dl_dimages(p) i(p) with j
 *   frozen (Eqs. Jaco1, TcofJaco1, DivTc):
 *   sum_c [T_c j_c B_c - D_c^T (T_c beta j_c B_c)], B_c = Pi_c^T dl_c.
 * 1 <= rays_per_side <= 64.  Scratch: 8 n_cams nx ny nz bytes (render), twice
 * that (gradient). */
int mc_voxel_scatter(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
                     const mc_params* params, double* j, mc_stats* stats, void* hip_stream);

int mc_voxel_render(const mc_grid* grid, const double* beta, int n_cams, const mc_camera* cams,
                    int rays_per_side, const double* j, double* images, void* hip_stream);

int mc_voxel_grad(const mc_grid* grid, const double* beta, int n_cams, const mc_camera* cams,
                  int rays_per_side, const double* j, const double* dl_dimages, const double* cam_weights,
                  double* grad_beta, void* hip_stream);

/* Recovery (Secs. 5.2, 6, 7).  All arrays are device arrays of doubles.
 * mc_voxel_conditioning: counts[c][k] = the sub-pixel rays (rays_per_side^2
 *   per pixel) of camera c whose length in voxel k exceeds 1e-9 of the
 *   shortest voxel edge (grazing rays are not counted); q[c][k] =
 *   1/counts (0 where no ray passes), the diagonal of the conditioning Q_c
 *   of Sec. 6 read as a normalisation by the number of rays (the reading
 *   that makes a voxel seen by many rays take a smaller step).  Either
 *   output may be NULL, not both.  Passed as cam_weights to mc_voxel_grad,
 *   q weights every camera's term of the gradient, Eq. (divCost1).
 * mc_regularizer: Psi = |W Lap beta|^2 (Sec. 6), Lap the 7-point Laplacian
 *   in voxel units with no flux through the domain boundary, W the diagonal
 *   of per-layer weights w_layer[iz] (NULL: 1).  value (nullable, one
 *   double) is overwritten with Psi; grad_beta (nullable) gets
 *   eta * 2 Lap^T W^T W Lap beta ADDED to it.
 * mc_image_residual: with r = mask (images - measured) (mask NULL: 1),
 *   dl_dimages = 2 mask r and *loss (nullable) = sum r^2: the data term of
 *   Eq. (Cost) and its image gradient.
 * mc_gd_step: beta = max(beta - delta grad, 0), Eq. (GD) on the
 *   non-negative set.
 * mc_camera_noise: Eq. (noise): scale = 2^10 / max(mask . images) over all
 *   cameras; out = floor(images scale + 0.4 normals + 1/2) clipped to
 *   [0, 1024]; normals are the caller's N(0,1) draws; *scale (nullable).
 * mc_recovery_error: out (HOST, two doubles) = delta_mass, eps of Sec. 7;
 *   waits for the stream.
 * mc_recover: n_outer surrogate iterations on beta (in/out): iteration q
 *   computes j with mc_voxel_scatter at the current beta and seed
 *   params->seed + q, then n_gd steps beta = max(beta - delta grad, 0) of
 *   E = sum |mask (i(beta | j) - measured)|^2 + eta Psi(beta), grad =
 *   2 sum_c Q_c J_c^T mask^2 (i - measured) + eta dPsi, Q_c = q of
 *   mc_voxel_conditioning (1/count) when conditioned = 1, the counts
 *   themselves (the passage's wording taken literally) when 2, 1 when 0.  cost (HOST,
 *   nullable, n_outer n_gd doubles) gets E before every step (one wait for
 *   the stream per step).  tally must be MC_TALLY_F64. */
int mc_voxel_conditioning(const mc_grid* grid, int n_cams, const mc_camera* cams, int rays_per_side,
                          double* counts, double* q, void* hip_stream);

int mc_regularizer(const mc_grid* grid, const double* beta, const double* w_layer, double eta,
                   double* grad_beta, double* value, void* hip_stream);

int mc_image_residual(int64_t n_pix, const double* images, const double* measured, const double* mask,
                      double* dl_dimages, double* loss, void* hip_stream);

int mc_gd_step(int64_t n, double* beta, const double* grad, double delta, void* hip_stream);

int mc_camera_noise(int64_t n_pix, const double* images, const double* mask, const double* normals,
                    double* out, double* scale, void* hip_stream);

int mc_recovery_error(int64_t n, const double* beta_hat, const double* beta_true, double* out,
                      void* hip_stream);

int mc_recover(const mc_grid* grid, double* beta, int n_cams, const mc_camera* cams, const mc_params* params,
               int rays_per_side, const double* measured, const double* mask, const double* w_layer,
               double eta, double delta, int n_gd, int n_outer, int conditioned, double* cost,
               void* hip_stream);

/* Test and diagnostics export: the first max_rec collisions of each of the
 * photons first_pid .. first_pid+count-1, for path-by-path comparison.
 * events: device array of count*max_rec mc_event (nullable if max_rec == 0);
 * pix: device array of count*max_rec*n_cams int32, the pixel row*width+col
 *   that each camera assigns to each recorded collision, or -1 (nullable);
 * paths: device array of count mc_path.  Slots past a photon's events are
 *   left untouched.  Always waits for the stream. */
typedef struct mc_event {
    double x, y, z;       /* collision point (km) */
    double w;             /* packet weight I_s at the collision, before the albedo factor */
    int32_t voxel;        /* voxel of the collision */
    int32_t pad_;
} mc_event;

enum { MC_FATE_TOP = 0, MC_FATE_BOTTOM = 1, MC_FATE_SIDE = 2, MC_FATE_RR = 3, MC_FATE_CAP = 4 };

typedef struct mc_path {
    int32_t n_events;     /* collisions of the photon */
    int32_t fate;         /* MC_FATE_* */
    double exit_pos[3];   /* exit point (fates TOP, BOTTOM, SIDE), else unspecified */
    double exit_dir[3];
    double exit_w;
} mc_path;

int mc_trace_paths(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
                   const mc_params* params, uint64_t first_pid, uint32_t count, uint32_t max_rec,
                   mc_event* events, int32_t* pix, mc_path* paths, void* hip_stream);

/* Diagnostic export: the gather capture.  mc_render with FP32 transport and
 * FP64 tallies (images as there) on at most max_waves wavefronts (a multiple
 * of 4; the launch may use fewer: *n_waves, host, gets the number), in which
 * wavefront w also stores, for its connection-walk steps first_step ..
 * first_step + n_steps - 1, the index into the library's copy of beta that
 * each of its 64 lanes asks for on that step (lanes with no ray, or in an
 * empty run of voxels, ask for index nx*ny*nz, which the walk's buffer
 * answers with zero and no memory access):
 * indices (device, max_waves * n_steps * 64 uint32) at
 * [(w * n_steps + step) * 64 + lane], left untouched where a wavefront took
 * fewer steps; wave_steps (device, max_waves uint32) gets each wavefront's
 * number of steps.  For measuring the walk's gathers against a replay of the
 * same addresses without the walk.  Waits for the stream when stats is
 * non-NULL.  MC_ERR_INVALID_ARG for grids whose walks take plain loads
 * (see MC_PLAIN_WALK_LOADS above). */
int mc_capture_gathers(const mc_grid* grid, const float* beta, int n_cams, const mc_camera* cams,
                       const mc_params* params, double* images, uint32_t first_step, uint32_t n_steps,
                       uint32_t max_waves, uint32_t* indices, uint32_t* wave_steps, uint32_t* n_waves,
                       mc_stats* stats, void* hip_stream);

/* Static description of a status code. */
const char* mc_error_string(int code);

/* Number of visible HIP devices (0 when none); never fails. */
int mc_device_count(void);

#ifdef __cplusplus
}
#endif
#endif /* MCRT_H */
