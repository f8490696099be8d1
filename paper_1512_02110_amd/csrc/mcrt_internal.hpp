// Host <-> kernel interface of the gfx950 renderer (private to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcrt.h"
#include "mcrt_device.hpp"

namespace mcrt {

// MODE_TAPE: gradient replay that writes rays with their gradient weight to
// the tape; MODE_RTAPE: render (image tallies) that also writes every ray
// with its local estimate to the tape, for a later gradient without replay.
// MODE_VOXEL: photon transport without local estimates that tallies the
// scattered power per voxel and camera (the voxelised model).
// MODE_BMC: backward Monte Carlo, packets traced from the camera pixels with
// the local estimate towards the sun.
enum {
    MODE_RENDER = 0, MODE_GRAD = 1, MODE_TRACE = 2, MODE_TAPE = 3, MODE_RTAPE = 4, MODE_VOXEL = 5, MODE_BMC = 6,
    MODE_MIXGRAD = 7
};
enum { TALLY_F64 = 0, TALLY_K32 = 1 };
enum {
    ST_PHOTONS = 0, ST_EVENTS, ST_LE, ST_VFREE, ST_VCONN,
    ST_TOP, ST_BOTTOM, ST_SIDE, ST_RR, ST_CAP, ST_N
};

// Camera as the host describes it, in double; the table is written to
// device memory by a kernel that receives it by value (no host buffer
// outlives the call).
struct HostCam {
    double pos[3];
    double R[9];
    double fx, fy, cx, cy;
    int32_t width, height;
    int64_t pix_off;
};

// Per-pixel normalisation table entry (double).
struct NormCam {
    double fx, fy, cx, cy;
    int32_t width, height;
    int64_t pix_off;
};

constexpr int CAM_CHUNK = 12;
struct CamChunk {
    int first, n;
    double dx, dy, dz;  // voxel edges, to express camera centres in voxel units
    HostCam c[CAM_CHUNK];
};

// Gradient tape of large grids.  The replay (MODE_TAPE) writes every
// connection ray with a non-zero weight to its wavefront's slice of the ray
// tape; a binning pass copies each ray into the bin of every
// gradient tile (at most TILE_VOX voxels) it crosses, and the deposit kernel
// accumulates each tile's bin in LDS.  A record holds the start of the ray
// and its pixel (ray tape) or camera (bins); direction and length are
// recomputed from the camera, so that a record fills whole 16-byte words.
template <typename Real>
struct alignas(16) TapeRec {
    uint32_t vox;       // start voxel: ix | iy << 11 | iz << 22
    uint32_t id;        // pixel (ray tape) or camera index (bins)
    Real fx, fy, fz;    // start fraction in the voxel
    Real a;             // gradient weight dL/di_p * norm_p * C
    Real ab;            // bins: a / beta(start voxel); records: 1, or 0 for an air
                        // collision of a mixture (bins: a / beta_aer or 0)
};

template <typename Real>
struct Tape {
    TapeRec<Real>* rec;       // rays: wavefront w owns slots [w rw, (w + 1) rw)
    uint32_t rw;              // ray slots per wavefront
    int w0;                   // first wavefront slice of a binning pass (block b: slice w0 + b)
    int scale_gw;             // records hold C (kept rays, replays): the binning passes take gw[pixel] * a
    uint32_t* wave_count;     // [wavefronts] rays written (more than rw: overflow)
    uint32_t* overflow;       // set when a wavefront ran out of slots
    TapeRec<Real>* brec;      // rays binned by tile
    uint32_t* tile_count;     // [n_tiles] records per tile
    // [n_tiles][n_slices]: records of tile t from the rays of block b of the
    // binning passes (block b: part b % split of wavefront slice
    // w0 + b / split); the scan turns them into first bin slots
    uint32_t* slice;
    int n_slices;             // binning blocks: split per wavefront slice
    int split;
    const uint32_t* bin_start; // [n_tiles] first slot of each tile's bin
    const uint32_t* tile_end;  // [n_tiles] end of each tile's bin
    int t_lo, t_hi;           // tiles binned by this pass
    int shx, shy, shz;        // tile edges are 2^sh voxels
    int n_tiles;
    Real itx, ity, itz;       // 1 / tile edges (exact)
    DevGrid<Real> T;          // grid of tiles (edges in km)
};

template <typename Real>
struct KArgs {
    DevGrid<Real> G;
    const Real* beta_le;        // the extinction the local estimates walk (beta, or
                                // the frozen-event render's evaluation field)
    int frozen;                 // frozen-event render: C *= beta_le / beta at the collision
    const Real* beta;           // the library's copy: n_vox values, then zeros
                                // (beta[n_vox] is fetched for empty voxels)
    // mixed precision (Real = double): the connection rays walk beta_w32, a
    // float copy of beta (then its zeros), on the grid G32 in float
    int walk32;
    const float* beta_w32;
    DevGrid<float> G32;
    int walk_buf;               // connection walks fetch through a buffer over the voxels
    const DevCam<Real>* cams;
    int n_cams;
    Real wsx, wsy, wsz;     // sun propagation direction
    Real albedo, g, rr;
    uint32_t max_events;
    uint64_t seed, pid0, n_photons;
    unsigned long long* work;   // photon counter (zeroed before launch)
    uint32_t fetch_block;       // photon ids a wavefront takes per fetch (set at launch)
    unsigned long long* stats;  // ST_N counters (zeroed before launch)
    double* img;                // raw local-estimate sums (F64 tally)
    double* img_m2;             // optional: raw sums of squared local estimates
    float* img32;               // [2 n_pix]: sum, compensation (K32 tally)
    const double* gw;           // dL/di * normalisation per pixel (gradient)
    double* grad;               // F64 gradient
    double* Lc;                 // voxel model: [voxel][lc_pitch] scattered power per camera
    int lc_pitch;               // cameras rounded up to a multiple of 8
    // air + aerosol mixture (render, MODE_MIXGRAD): beta is air + sig * aer
    const double* mix_air;      // nullptr: one constituent
    const double* mix_aer;      // aerosol field of the reference channel
    double mix_sig;             // aerosol cross-section ratio of the channel
    int mix_full;               // MODE_MIXGRAD: 1 full gradient, 0 surrogate
    double* mix_evs;            // full gradient: per lane, the first mix_evcap collisions' sums of a
    double* mix_rows;           // full gradient by the tape replay: per photon, those sums and the rest's
    uint32_t mix_evcap;
    // the word a voxel of an empty run reads: beta[air_base + iz * air_step]
    // (n_vox and 0: the zero; the air column and 1: air by height)
    uint32_t air_base, air_step;
    const HostCam* hcams;       // backward MC: cameras in double, absolute positions
    uint32_t n_pp;              // backward MC: packets per pixel
    float* grad32;              // [2 n_vox] (K32 gradient)
    int64_t n_pix, n_vox;
    // occupancy bitmask of beta > 0: bit c covers voxels [c 2^msh, (c+1) 2^msh)
    const uint32_t* mask;
    int msh, mask_words;
    int grad_lds;               // gradient privatised in LDS (small grids)
    int tape;                   // gradient through the tape (large grids)
    Tape<Real> tp;
    // gather capture (a diagnostic of the FP32 render): wavefront w stores the
    // extinction index each lane loads on connection-walk steps
    // cap_first .. cap_first + cap_steps - 1 of the wavefront at
    // capture[(w cap_steps + step) 64 + lane], and its number of steps at
    // capture_steps[w]
    uint32_t* capture;
    uint32_t* capture_steps;
    uint32_t cap_first, cap_steps;
    // trace
    uint64_t first_pid;
    uint32_t trace_count, max_rec;
    mc_event* ev;
    int32_t* pix;
    mc_path* paths;
};

// LDS budget of the occupancy bitmask: 16 KB (131072 bits) for FP32 and
// mixed-precision transport, so that four 256-thread blocks fit a CU's 160 KB
// of LDS; 32 KB for FP64 transport (two blocks per CU, register bound).
constexpr int MASK_WORDS_FP32 = 4096;
constexpr int MASK_WORDS = 8192;
constexpr int TILE_VOX = 16384;   // voxels of a gradient tile
// LDS slots of a tile in the deposit kernel: the tile with one padding
// column after every row and one padding row after every layer,
// (nx + 1)(ny + 1)nz <= TILE_LDS (145 KB for 16 x 16 x 64).  A walk step that
// rounding carries across the tile's x or y face lands in a padding slot,
// which is never flushed, instead of in another voxel of the tile.
constexpr int TILE_LDS = 18560;
constexpr int MAX_TAPE_TILES = 8192;  // per-tile counters of the binning pass: up to 104 KB of LDS
constexpr int BIN_LDS_CAMS = 2048;    // camera pixel offsets the binning pass keeps in LDS
constexpr int BIN_GROUP_TILES = 4096; // tiles per scatter pass (3 LDS words each)
// Binning blocks of a pass: at least BIN_BLOCKS_PER_CU per compute unit
// (a slice of the ray tape split over up to BIN_SPLIT_MAX blocks): a pass of
// a few hundred wavefront slices would otherwise fill a fraction of the GPU,
// and more, smaller blocks shorten the launch's last round.
constexpr int BIN_BLOCKS_PER_CU = 32;
constexpr int BIN_SPLIT_MAX = 64;
constexpr int SCAN_BLOCK = 256;
constexpr int DEPOSIT_BLOCK = 1024;
constexpr int DEP_LDS_CAMS = 256;     // camera centres the deposit keeps in LDS
// Deposit items per compute unit and group of tiles.  A deposit block takes a
// whole CU (its LDS copy of a tile), so the launch runs in rounds of n_cu
// blocks; items of about 1/DEP_ITEMS_PER_CU of a CU's share, started largest
// first, keep the last round short (measured against two items per CU in
// launch order: the gradient 10-16% faster on the 64^3, 128^3 and
// 256x256x128 workloads; 8 and 32 per CU were up to 3% slower than 16).
constexpr int DEP_ITEMS_PER_CU = 16;

// Work item of the deposit kernel: slots [lo, hi) of one tile's range.
struct DepositItem {
    int32_t tile;
    uint32_t lo, hi;
    uint32_t pad_;
};
constexpr int64_t GRAD_LDS_BYTES = 64 * 1024;  // dynamic LDS budget of a privatised gradient

constexpr int BLOCK = 256;
constexpr int BETA_PAD = 64;  // zeros after the library's copy of beta

// Launchers (mcrt_kernels.hip).
template <typename Real>
hipError_t launch_write_cams(const CamChunk& chunk, DevCam<Real>* dev, NormCam* norm, hipStream_t s);
template <typename Real>
hipError_t launch_transport(const KArgs<Real>& a, int mode, int tally, int grid, hipStream_t s);
hipError_t launch_capture(const KArgs<float>& a, int grid, hipStream_t s);
template <typename Real>
hipError_t transport_occupancy(const KArgs<Real>& a, int mode, int tally, int* blocks_per_cu);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t s);
hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, hipStream_t s);
hipError_t launch_normalize(double* img, const NormCam* cams, int n_cams, int64_t n_pix, double base, int power,
                            hipStream_t s);
hipError_t launch_grad_weights(double* gw, const double* dl, const NormCam* cams, int n_cams, int64_t n_pix,
                               double base, hipStream_t s);
hipError_t launch_kahan_reduce(double* out, const float* pairs, int64_t n, hipStream_t s);
template <typename Real>
hipError_t launch_build_mask(const KArgs<Real>& a, uint32_t* mask, hipStream_t s);
template <typename Real>
hipError_t launch_build_mask_aer(const KArgs<Real>& a, uint32_t* mask, hipStream_t s);
template <typename Real>
hipError_t launch_air_column(const double* air, int64_t n_vox, int64_t nxy, int nz, Real* col, uint32_t* flag,
                             hipStream_t s);
template <typename Real>
hipError_t launch_mix_path(const KArgs<Real>& a, int grid, hipStream_t s);
template <typename Real>
hipError_t launch_mix_total(Real* beta, const double* air, const double* aer, double sig, int64_t n, int64_t pad,
                            hipStream_t s);
template <typename Real>
hipError_t launch_bin(const KArgs<Real>& a, bool scatter, hipStream_t s);
template <typename Real>
hipError_t launch_bin_scan(const KArgs<Real>& a, hipStream_t s);
template <typename Real>
hipError_t launch_deposit(const KArgs<Real>& a, int tally, const DepositItem* items, int n_items, hipStream_t s);
template <typename Real>
hipError_t launch_voxel_finish(double* j, const double* L, int pitch, const Real* beta, int n_cams, int64_t n_vox,
                               double base, hipStream_t s);

// Voxelised model, deterministic part (mcrt_voxel.hip): FP64 throughout.
// Cameras as HostCam (double), uploaded by k_vox_cams from kernel arguments.
struct VoxArgs {
    int nx, ny, nz;
    double dx, dy, dz;
    int64_t n_vox;
    const double* beta;
    const HostCam* cams;
    int n_cams;
    int n_side;                 // sub-pixel rays per side (n_side^2 per pixel)
    int64_t n_pix;
    double* T;                  // [camera][voxel] transmittance to the camera
    const double* j;            // [camera][voxel]
    double* images;
    const double* dl;
    double* B;                  // [camera][voxel] back-projected image gradient
    const double* q;            // [camera][voxel] weights of the camera terms (nullable)
    double* grad;
};
hipError_t launch_vox_cams(const CamChunk& chunk, HostCam* dev, hipStream_t s);
hipError_t launch_vox_transmittance(const VoxArgs& a, hipStream_t s);
hipError_t launch_vox_project(const VoxArgs& a, hipStream_t s);
hipError_t launch_vox_backproject(const VoxArgs& a, hipStream_t s);
hipError_t launch_vox_los_adjoint(const VoxArgs& a, hipStream_t s);
hipError_t launch_vox_ray_counts(const VoxArgs& a, double* counts, hipStream_t s);
hipError_t launch_vox_invert(double* x, int64_t n, hipStream_t s);
hipError_t launch_reg(int nx, int ny, int nz, const double* beta, const double* w_layer, double eta, double* r,
                      double* grad, double* value, hipStream_t s);
hipError_t launch_image_residual(int64_t n, const double* img, const double* meas, const double* mask, double* dl,
                                 double* loss, hipStream_t s);
hipError_t launch_gd_step(int64_t n, double* beta, const double* g, double delta, hipStream_t s);
hipError_t launch_camera_noise(int64_t n, const double* img, const double* mask, const double* normals,
                               unsigned long long* mx, double* out, double* scale_out, hipStream_t s);
hipError_t launch_recovery_sums(int64_t n, const double* b, const double* t, double* acc, hipStream_t s);
hipError_t launch_d2f(int64_t n, const double* in, float* out, hipStream_t s);


}  // namespace mcrt
