// Host <-> kernel interface of the gfx950 renderer (private to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcrt.h"
#include "mcrt_device.hpp"

namespace mcrt {

enum { MODE_RENDER = 0, MODE_GRAD = 1, MODE_TRACE = 2 };
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

// Gradient tape of large grids.  The grid is cut into tiles of at most
// TILE_VOX voxels; the replay writes one record per connection ray and tile
// the ray crosses, into that tile's slot range [off, off + cap) of the
// structure-of-arrays below, and the deposit kernel then accumulates each
// tile's records in LDS.  A slot whose weight a is 0 is empty.
template <typename Real>
struct Tape {
    uint32_t* vox;            // start voxel: ix | iy << 11 | iz << 22
    Real *fx, *fy, *fz;       // start fraction in the voxel
    Real *vx, *vy, *vz;       // unit direction to the camera
    Real* r;                  // length to the camera (km)
    Real* a;                  // gradient weight dL/di_p * norm_p * C
    uint32_t* count;          // [n_tiles] slots handed out (may exceed cap)
    const uint32_t* off;      // [n_tiles]
    const uint32_t* cap;      // [n_tiles]
    uint32_t* overflow;       // set when a tile ran out of slots
    uint32_t block;           // slots a wavefront reserves at a time
    int tx, ty, tz, n_tiles;  // tile edges in voxels
    Real itx, ity, itz;       // 1 / tile edges
    DevGrid<Real> T;          // grid of tiles (edges in km)
};

template <typename Real>
struct KArgs {
    DevGrid<Real> G;
    const Real* beta;
    const DevCam<Real>* cams;
    int n_cams;
    Real wsx, wsy, wsz;     // sun propagation direction
    Real albedo, g, rr;
    uint32_t max_events;
    uint64_t seed, pid0, n_photons;
    unsigned long long* work;   // photon counter (zeroed before launch)
    unsigned long long* stats;  // ST_N counters (zeroed before launch)
    double* img;                // raw local-estimate sums (F64 tally)
    double* img_m2;             // optional: raw sums of squared local estimates
    float* img32;               // [2 n_pix]: sum, compensation (K32 tally)
    const double* gw;           // dL/di * normalisation per pixel (gradient)
    double* grad;               // F64 gradient
    float* grad32;              // [2 n_vox] (K32 gradient)
    int64_t n_pix, n_vox;
    // occupancy bitmask of beta > 0 over cells of 2^msh voxels per axis
    const uint32_t* mask;
    int mshx, mshy, mshz, mncx, mncy, mask_words, mask_fine;
    int grad_lds;               // gradient privatised in LDS (small grids)
    int tape;                   // gradient through the tape (large grids)
    Tape<Real> tp;
    // trace
    uint64_t first_pid;
    uint32_t trace_count, max_rec;
    mc_event* ev;
    int32_t* pix;
    mc_path* paths;
};

constexpr int MASK_WORDS = 8192;  // 32 KB of LDS: up to 262144 cells
constexpr int TILE_VOX = 16384;   // voxels of a gradient tile (128 KB of FP64 LDS)
constexpr int MAX_TAPE_TILES = 640;
constexpr int DEPOSIT_BLOCK = 1024;

// Work item of the deposit kernel: slots [lo, hi) of one tile's range.
struct DepositItem {
    int32_t tile;
    uint32_t lo, hi;
    uint32_t pad_;
};
constexpr int64_t GRAD_LDS_BYTES = 64 * 1024;  // dynamic LDS budget of a privatised gradient

constexpr int BLOCK = 256;

// Launchers (mcrt_kernels.hip).
template <typename Real>
hipError_t launch_write_cams(const CamChunk& chunk, DevCam<Real>* dev, NormCam* norm, hipStream_t s);
template <typename Real>
hipError_t launch_transport(const KArgs<Real>& a, int mode, int tally, int grid, hipStream_t s);
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
hipError_t launch_build_mask(const KArgs<Real>& a, uint32_t* mask, int ncz, hipStream_t s);
template <typename Real>
hipError_t launch_deposit(const KArgs<Real>& a, int tally, const DepositItem* items, int n_items, hipStream_t s);


}  // namespace mcrt
