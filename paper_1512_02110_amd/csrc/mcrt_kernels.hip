// Kernels of the gfx950 renderer.
//
// The photon life cycle is that of Sec. 2.1.2 (steps i-vi): launch at the
// top of the domain along the sun direction, free flight by voxel walk to the
// optical depth drawn by Eq. (taurand) (Eq. MCextinct solved exactly inside
// each voxel), albedo weighting with Russian roulette, HG scattering
// (Eq. thetaHG); at every collision the local estimate of Sec. 2.1.3,
// Eq. (fle), to every camera that sees the collision, attenuated by the
// transmittance of the connecting ray (Eqs. beer-lambert, tc).
//
// k_render (forward and gradient): persistent wavefronts with two phases.
//   * Photon phase: each lane owns one photon; a lane whose photon ended takes
//     the next photon id (the lanes of a wavefront take a block of ids with
//     one atomic).  Lanes fly to their next collision and, for every camera
//     that sees it, push a local-estimate job (start voxel and fraction,
//     direction and length to the camera, prefactor, pixel) into the
//     wavefront's LDS queue, compacted with ballot/prefix counts.
//   * Job phase: the 64 lanes walk connection rays taken from the queue.
//     Lanes that finish are refilled together once 16 are idle, so the walk
//     runs with nearly full wavefronts whatever the ray lengths and the
//     number of cameras each collision is visible from.  A lane keeps an
//     unfinished ray across photon phases.
// MODE_GRAD replays the same photons; a finished connection ray with
// contribution C to pixel p scatters the surrogate gradient (Sec. 5.2,
// Eqs. Jaco1, TcofJaco1, DivTc for one event): grad[k_e] += a / beta(k_e)
// and, walking the ray again, grad[m] -= a l(m), with a = dL/di_p norm_p C.
// Small grids accumulate this in a per-workgroup LDS copy of the gradient.
// Large grids replay in MODE_TAPE instead (or keep the rays of the render,
// MODE_RTAPE): the finished ray goes to a tape, k_bin copies it into the bin
// of every gradient tile it crosses, and k_deposit accumulates every tile's
// bin in LDS.  The gradients of an air + aerosol mixture use the same
// replay and bins.  A device-scope atomic add
// per voxel crossing would run at the memory-side atomic rate, far below the
// walk.
//
// k_trace: one photon per lane, the same transport, recording events.
#include <algorithm>

#include "mcrt_internal.hpp"

namespace mcrt {

constexpr int WAVE = 64;
constexpr uint32_t QCAP = 128;     // local-estimate jobs per wavefront queue
// A wavefront's connection walks are refilled from its queue once this many
// lanes are idle (measured on the 64^3 and 128^3 workloads: 32 is 2% faster
// than 16 or 24, 8 and 12 are slower); the deposit of the gradient likewise.
constexpr uint32_t REFILL_IDLE = 32;
constexpr uint32_t DEP_REFILL_IDLE = 32;

// Photon packet: voxel-local position (voxel i, fraction f of the voxel
// edge), direction, weight and the optical depth still to fly.
template <typename Real>
struct Photon {
    int ix, iy, iz;
    Real fx, fy, fz;
    Real wx, wy, wz;
    Real weight;
    Real taustar;
    Real t_exit;  // ray parameter at which the last flight left the domain
    uint32_t s;   // collisions so far
    uint64_t pid;
    int air;      // particle of the last collision: 1 air, 0 aerosol (mixture)
};

// Absolute coordinate (km) of a voxel-local position.
template <typename Real>
__device__ __forceinline__ double absolute(int i, Real f, Real d) {
    return ((double)i + (double)f) * (double)d;
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long mask) {
    return (uint32_t)__popcll(mask & __lanemask_lt());
}

// Photon ids for the lanes in `need`, in order, from the wavefront's pool
// [pool_next, pool_end), which is refilled `block` ids at a time with one
// atomic on the global counter (a returning device atomic takes
// microseconds; one per photon phase would stall every phase).  Called by
// the whole wavefront, so that the pool stays uniform.  One refill must
// cover every lane that still needs an id, so a block holds at least WAVE
// ids; within that, the launch sets it so that every wavefront fetches about
// 32 times (at most 256 ids): a launch ends with its slowest wavefront, and
// a few large blocks per wavefront leave the others idle at the end.
constexpr uint32_t FETCH_BLOCK_MAX = 256;

__device__ __forceinline__ uint64_t wave_fetch(unsigned long long* work, uint32_t block, unsigned long long need,
                                               uint64_t& pool_next, uint64_t& pool_end) {
    const uint32_t n = (uint32_t)__popcll(need);
    const uint32_t rank = lanes_below(need);
    const uint64_t left = pool_end - pool_next;
    const uint32_t avail = left < n ? (uint32_t)left : n;
    uint64_t id = pool_next + rank;
    if (avail < n) {
        unsigned long long base = 0;
        if (__lane_id() == 0) base = atomicAdd(work, (unsigned long long)block);
        const unsigned lo = __shfl((unsigned)base, 0);
        const unsigned hi = __shfl((unsigned)(base >> 32), 0);
        pool_next = ((uint64_t)hi << 32) | lo;
        pool_end = pool_next + block;
        if (rank >= avail) id = pool_next + (rank - avail);
        pool_next += n - avail;
    } else {
        pool_next += n;
    }
    return id;
}

// Error-free FP32 accumulation: the sum goes to pair[0], the rounding error
// of the conversion and of the atomic add to pair[1].  The add's error is
// recovered from the value the atomic returned (TwoSum, Knuth).
__device__ __forceinline__ void k32_add(float* pair, double x) {
    const float xf = (float)x;
    const float rconv = (float)(x - (double)xf);
    const float old = atomicAdd(pair, xf);
    const float s = old + xf;
    const float bp = s - old;
    const float err = (old - (s - bp)) + (xf - bp);
    const float c = err + rconv;
    if (c != 0.0f) atomicAdd(pair + 1, c);
}

template <int TALLY>
__device__ __forceinline__ void tally_f64(double* base, float* base32, int64_t i, double x) {
    if (TALLY == TALLY_F64) {
        unsafeAtomicAdd(base + i, x);
    } else {
        k32_add(base32 + 2 * i, x);
    }
}

// Gradient deposit: into the block's LDS copy of the whole gradient when the
// grid is small enough to be privatised (flushed once at the end of the
// kernel), else straight to the device array.
template <typename Real, int TALLY>
__device__ __forceinline__ void grad_add(const KArgs<Real>& A, double* lds_grad, int64_t k, double x) {
    if (lds_grad) {
        atomicAdd(lds_grad + k, x);
    } else {
        tally_f64<TALLY>(A.grad, A.grad32, k, x);
    }
}

// ---------------------------------------------------------------------------
// Voxel walk in registers.  Along the unit direction w from the voxel-local
// point (i, f), the next crossing on axis a is t_a = r_a g_a with
// g_a = d_a / w_a and r_a = (index of the next face counted from the start
// voxel's lower face) - f_a; after a crossing on axis a, r_a moves by the step
// s_a and t_a is recomputed (no accumulated error).  Axes with a zero
// component have r = 1, g = inf.  Ties go to the lowest axis.
//
// These helpers only ever choose between a register value and a constant:
// a choice between two fields reached through a reference is turned by the
// compiler into a choice between their addresses, which would move the walk
// to scratch memory.
template <typename Real>
struct WalkRegs {
    int ix, iy, iz, k;
    int sx, sy, sz;
    int kx, ky, kz;      // index step of a crossing on each axis
    Real sfx, sfy, sfz;  // the steps as Real
    Real rx, ry, rz;
    Real gx, gy, gz;
    Real tx, ty, tz;
    Real t;              // entry parameter of the current voxel
};

template <typename Real>
__device__ __forceinline__ void walk_axis(Real f, Real w, Real d, int& s, Real& sf, Real& r, Real& g, Real& tn) {
    // components below `tiny` count as zero so that g stays finite
    const Real tiny = sizeof(Real) == 4 ? (Real)1e-20f : (Real)1e-200;
    s = w > tiny ? 1 : (w < -tiny ? -1 : 0);
    sf = (Real)s;
    const Real fc = f < (Real)0 ? (Real)0 : (f > (Real)1 ? (Real)1 : f);
    if (s != 0) {
        g = d / w;
        r = s > 0 ? (Real)1 - fc : -fc;
    } else {
        g = (Real)INFINITY;
        r = (Real)1;
    }
    tn = r * g;
}

// Returns false when the walk cannot start (non-finite fraction or no usable
// direction component); the caller then treats it as having left the
// domain.  Otherwise every crossing advances one index on an axis with a
// non-zero step, so a walk ends after at most nx + ny + nz crossings.
template <typename Real>
__device__ __forceinline__ bool walk_begin(WalkRegs<Real>& W, const DevGrid<Real>& G, int ix, int iy, int iz, Real fx,
                                           Real fy, Real fz, Real wx, Real wy, Real wz) {
    W.ix = ix;
    W.iy = iy;
    W.iz = iz;
    W.k = ix + G.nx * iy + G.nxy * iz;
    walk_axis(fx, wx, G.dx, W.sx, W.sfx, W.rx, W.gx, W.tx);
    walk_axis(fy, wy, G.dy, W.sy, W.sfy, W.ry, W.gy, W.ty);
    walk_axis(fz, wz, G.dz, W.sz, W.sfz, W.rz, W.gz, W.tz);
    W.kx = W.sx;
    W.ky = W.sy * G.nx;
    W.kz = W.sz * G.nxy;
    W.t = (Real)0;
    const bool finite_f = fabs(fx) < (Real)4 && fabs(fy) < (Real)4 && fabs(fz) < (Real)4;
    return finite_f && (W.sx | W.sy | W.sz) != 0;
}

// Parameter of the next crossing; cx/cy/cz tell on which axis it is.
template <typename Real>
__device__ __forceinline__ Real walk_next(const WalkRegs<Real>& W, bool& cx, bool& cy, bool& cz) {
    cx = (W.tx <= W.ty) && (W.tx <= W.tz);
    cy = !cx && (W.ty <= W.tz);
    cz = !cx && !cy;
    return fmin(W.tx, fmin(W.ty, W.tz));
}

// Cross the face at tn; returns true when the walk left the domain (the
// state is then only meaningful for the indices).
template <typename Real>
__device__ __forceinline__ bool walk_cross(WalkRegs<Real>& W, const DevGrid<Real>& G, Real tn, bool cx, bool cy,
                                           bool cz) {
    W.t = tn;
    W.ix += cx ? W.sx : 0;
    W.iy += cy ? W.sy : 0;
    W.iz += cz ? W.sz : 0;
    W.k += (cx ? W.kx : 0) + (cy ? W.ky : 0) + (cz ? W.kz : 0);
    W.rx += cx ? W.sfx : (Real)0;
    W.ry += cy ? W.sfy : (Real)0;
    W.rz += cz ? W.sfz : (Real)0;
    W.tx = W.rx * W.gx;
    W.ty = W.ry * W.gy;
    W.tz = W.rz * W.gz;
    return (unsigned)W.ix >= (unsigned)G.nx || (unsigned)W.iy >= (unsigned)G.ny || (unsigned)W.iz >= (unsigned)G.nz;
}

// Fraction along one axis, relative to the current voxel, of the point at
// parameter tp of a walk that started at fraction f0, clamped to [0, 1].
template <typename Real>
__device__ __forceinline__ Real walk_frac(Real f0, Real sf, Real r, Real w, Real id, Real tp) {
    // faces crossed so far along the axis (signed) = r - r0 with r0 = 1 - f0
    // (s > 0) or -f0 (s < 0); the new fraction is f0 + tp w / d - crossed
    const Real fc = f0 < (Real)0 ? (Real)0 : (f0 > (Real)1 ? (Real)1 : f0);
    const Real r0 = sf > (Real)0 ? (Real)1 - fc : (sf < (Real)0 ? -fc : (Real)1);
    const Real crossed = r - r0;
    Real q = fc + tp * w * id - crossed;
    q = q < (Real)0 ? (Real)0 : q;
    return q > (Real)1 ? (Real)1 : q;
}

// Occupancy of voxel k in the bitmask of runs of 2^msh consecutive voxels
// that hold a non-zero extinction: an empty voxel contributes nothing to any
// optical depth, so its extinction need not be fetched.  (A run of voxels
// along x, possibly wrapping to the next row, costs one shift to index.)
template <typename Real>
__device__ __forceinline__ bool occupied(const KArgs<Real>& A, const uint32_t* mask, int k) {
    const uint32_t cell = (uint32_t)k >> A.msh;
    return (mask[cell >> 5] >> (cell & 31u)) & 1u;
}

// Where a voxel of an empty run (layer iz) reads its extinction: the zero
// after the last voxel, or, for a mixture whose air depends on the height
// only (the runs then mark the aerosol), the air column's value for the
// layer.  Either way every lane reads one of a few words (no gather).
template <typename Real>
__device__ __forceinline__ uint32_t empty_index(const KArgs<Real>& A, int iz) {
    return A.air_base + (uint32_t)iz * A.air_step;
}

// Extinction of voxel k (layer iz), read from the empty-run word when its
// run is empty (no mask: always gathered).
template <typename Real>
__device__ __forceinline__ Real beta_at(const KArgs<Real>& A, const uint32_t* mask, int k, int iz) {
    if (mask && !occupied(A, mask, k)) return A.air_step ? A.beta[empty_index(A, iz)] : (Real)0;
    return A.beta[k];
}

// Structured buffer loads (element index times the descriptor's stride): an
// index at or past the descriptor's record count returns zero and makes no
// memory access.
__device__ float buf_load_f32(__amdgpu_buffer_rsrc_t rsrc, int index, int offset, int soffset, int aux) __asm(
    "llvm.amdgcn.struct.ptr.buffer.load.f32");
__device__ double buf_load_f64(__amdgpu_buffer_rsrc_t rsrc, int index, int offset, int soffset, int aux) __asm(
    "llvm.amdgcn.struct.ptr.buffer.load.f64");

// What the walk of a connection ray reads: the extinction it walks (the
// library's copy of beta followed by zeros and, for a mixture, the air
// column), the grid, both in the walk's precision W, and the occupancy
// bitmask's run shift.  W is the transport precision, except in mixed
// precision (photon state in FP64), where the connection rays walk a float
// copy of beta on the grid in float.
//
// The render's and the tape's walks fetch through `rs`, a buffer over the
// n_vox voxels only: a lane whose ray has ended or which is in an empty run
// asks for index n_vox and gets zero without a memory access (with a plain
// load every such lane reads the shared zero word, about a quarter of the
// vector-memory accesses of the render).  The kernels whose walks read an air
// column (AIRZ) use plain loads; the host also launches those, with the air
// column at the zero word, for grids too large for a buffer.
template <typename W>
struct WalkCtx {
    const W* beta;
    DevGrid<W> G;
    uint32_t n_vox;
    int msh;
    uint32_t air_base, air_step;
    __amdgpu_buffer_rsrc_t rs;
    // where a voxel of an empty run in layer iz reads its extinction
    __device__ __forceinline__ uint32_t empty(int iz) const { return air_base + (uint32_t)iz * air_step; }
    __device__ __forceinline__ bool occ(const uint32_t* mask, int k) const {
        const uint32_t cell = (uint32_t)k >> msh;
        return (mask[cell >> 5] >> (cell & 31u)) & 1u;
    }
    // the extinction of voxel k (layer iz) as one unconditional load, so that
    // the loaded register can stay in flight across a step without a select
    __device__ __forceinline__ W load(const uint32_t* mask, int k, int iz) const {
        return beta[occ(mask, k) ? (uint32_t)k : empty(iz)];
    }
    // the extinction at index i <= n_vox: through the buffer (BUF) or a plain load
    template <bool BUF>
    __device__ __forceinline__ W fetch(uint32_t i) const {
        if constexpr (!BUF) {
            return beta[i];
        } else if constexpr (sizeof(W) == 4) {
            return buf_load_f32(rs, (int)i, 0, 0, 0);
        } else {
            return buf_load_f64(rs, (int)i, 0, 0, 0);
        }
    }
};

template <typename Real, bool W32>
struct WalkPrec {
    using type = Real;
};
template <typename Real>
struct WalkPrec<Real, true> {
    using type = float;
};

template <typename Real, bool W32>
__device__ __forceinline__ WalkCtx<typename WalkPrec<Real, W32>::type> walk_ctx(const KArgs<Real>& A) {
    WalkCtx<typename WalkPrec<Real, W32>::type> C;
    if constexpr (W32) {
        C.beta = A.beta_w32;
        C.G = A.G32;
    } else {
        C.beta = A.beta_le;
        C.G = A.G;
    }
    C.n_vox = (uint32_t)A.n_vox;
    // stride sizeof(W), n_vox records; the last dword sets the 32-bit data
    // format that untyped buffer loads of CDNA expect
    C.rs = __builtin_amdgcn_make_buffer_rsrc((void*)C.beta, (short)sizeof(C.beta[0]), (int)C.n_vox, 0x00020000);
    C.msh = A.msh;
    C.air_base = A.air_base;
    C.air_step = A.air_step;
    return C;
}

// ---------------------------------------------------------------------------
// Photon transport steps.

template <typename Real>
__device__ __forceinline__ void launch_photon(const KArgs<Real>& A, uint64_t pid, Photon<Real>& ph) {
    const uint4 r = draw(A.seed, pid, 0u);
    // uniform point of the top face, in voxel units
    const Real px = uniform01<Real>(r.x) * (Real)A.G.nx;
    const Real py = uniform01<Real>(r.y) * (Real)A.G.ny;
    const int ix = (int)m_floor(px), iy = (int)m_floor(py);
    ph.ix = ix < A.G.nx - 1 ? ix : A.G.nx - 1;
    ph.iy = iy < A.G.ny - 1 ? iy : A.G.ny - 1;
    ph.iz = A.G.nz - 1;
    ph.fx = px - (Real)ph.ix;
    ph.fy = py - (Real)ph.iy;
    ph.fz = (Real)1;
    ph.wx = A.wsx;
    ph.wy = A.wsy;
    ph.wz = A.wsz;
    ph.weight = (Real)1;
    ph.taustar = -m_log((Real)1 - uniform01<Real>(r.z));
    ph.t_exit = (Real)0;
    ph.s = 0;
    ph.pid = pid;
    ph.air = 0;
}

// Steps (ii)-(iii): returns 0 on a collision (position and voxel updated),
// 1 + face code (0 top, 1 bottom, 2 side) when the photon left the domain
// (position unchanged, t_exit set), or FLIGHT_GOES_ON when `budget` voxels
// were crossed without either: the photon then stands at the entry point of
// its current voxel with the optical depth still to fly, and the next call
// continues the flight.  (A wavefront steps all its photons' flights
// together; a budget keeps the lanes whose flights are short from waiting
// for the longest one.)
constexpr int FLIGHT_GOES_ON = 4;
constexpr uint32_t FLIGHT_BUDGET = 32;

//
// DEP: also subtract dep times the length flown in every voxel from grad
// (the free-flight score of the full mixture gradient).
template <typename Real, bool DEP = false>
__device__ __forceinline__ int free_flight(const KArgs<Real>& A, const uint32_t* mask, Photon<Real>& ph,
                                           uint64_t& vfree, uint32_t budget, double dep = 0.0,
                                           double* grad = nullptr) {
    WalkRegs<Real> W;
    const Real f0x = ph.fx, f0y = ph.fy, f0z = ph.fz;
    const Real wx = ph.wx, wy = ph.wy, wz = ph.wz;
    const Real taustar = ph.taustar;
    if (!walk_begin(W, A.G, ph.ix, ph.iy, ph.iz, f0x, f0y, f0z, wx, wy, wz)) {
        ph.t_exit = (Real)0;
        return 3;
    }
    Real tau = (Real)0, tc = (Real)0;
    Real b = beta_at(A, mask, W.k, W.iz);
    uint32_t steps = 0;
    int left = 0;
    for (;;) {
        ++steps;
        bool cx, cy, cz;
        const Real tn = walk_next(W, cx, cy, cz);
        const Real seg = tn - W.t;
        if (b > (Real)0 && tau + b * seg >= taustar) {
            tc = W.t + (taustar - tau) / b;
            if (DEP && dep != 0.0) unsafeAtomicAdd(grad + W.k, -dep * (double)(tc - W.t));
            break;
        }
        if (DEP && dep != 0.0) unsafeAtomicAdd(grad + W.k, -dep * (double)seg);
        tau += b * seg;
        const bool out = walk_cross(W, A.G, tn, cx, cy, cz);
        if (out) {
            left = cz ? (W.sz > 0 ? 1 : 2) : 3;
            break;
        }
        if (steps >= budget) {
            left = FLIGHT_GOES_ON;
            tc = W.t;
            break;
        }
        b = beta_at(A, mask, W.k, W.iz);
    }
    vfree += steps;
    if (left == 0 || left == FLIGHT_GOES_ON) {
        ph.fx = walk_frac(f0x, W.sfx, W.rx, wx, A.G.idx, tc);
        ph.fy = walk_frac(f0y, W.sfy, W.ry, wy, A.G.idy, tc);
        ph.fz = walk_frac(f0z, W.sfz, W.rz, wz, A.G.idz, tc);
        ph.ix = W.ix;
        ph.iy = W.iy;
        ph.iz = W.iz;
        if (left == FLIGHT_GOES_ON) ph.taustar = taustar - tau;
    } else {
        ph.t_exit = W.t;
    }
    return left;
}

// Local-estimate geometry of the collision at (i, f) for one camera
// (Sec. 2.1.3): false when the camera does not see the point.  Otherwise
// returns the pixel, the unit direction to the camera, its length r and
// albedo * I_s * P(angle) / r^2.
template <typename Real>
__device__ __forceinline__ bool le_geometry(const KArgs<Real>& A, const DevCam<Real>& cam, int ix, int iy, int iz,
                                            Real fx, Real fy, Real fz, Real wx, Real wy, Real wz, Real weight,
                                            int air, int64_t& pix, int& local_pix, Real& vx, Real& vy, Real& vz,
                                            Real& r, Real& pre) {
    // X - X_c from voxel-local parts (the integer differences are exact),
    // projected in FP64 for either transport precision: the pixel and the
    // cull are discrete choices, made in double from the collision point
    const double dx = ((double)(ix - cam.icx) + ((double)fx - cam.pfcx)) * A.G.ddx;
    const double dy = ((double)(iy - cam.icy) + ((double)fy - cam.pfcy)) * A.G.ddy;
    const double dz = ((double)(iz - cam.icz) + ((double)fz - cam.pfcz)) * A.G.ddz;
    const double qz = cam.R[6] * dx + cam.R[7] * dy + cam.R[8] * dz;
    if (!(qz > 0.0)) return false;
    const double qx = cam.R[0] * dx + cam.R[1] * dy + cam.R[2] * dz;
    const double qy = cam.R[3] * dx + cam.R[4] * dy + cam.R[5] * dz;
    const double u = cam.fx * qx / qz + cam.cx;
    const double v = cam.fy * qy / qz + cam.cy;
    if (!(u >= 0.0 && u < cam.fw && v >= 0.0 && v < cam.fh)) return false;
    const double r2d = dx * dx + dy * dy + dz * dz;
    if (r2d < 1e-12) return false;
    local_pix = (int)v * cam.width + (int)u;
    pix = (int64_t)cam.pix_off + local_pix;
    // the rest in the transport precision
    const Real r2 = (Real)r2d;
    r = m_sqrt(r2);
    const Real ir = (Real)1 / r;
    vx = -(Real)dx * ir;
    vy = -(Real)dy * ir;
    vz = -(Real)dz * ir;
    const Real cosang = wx * vx + wy * vy + wz * vz;
    // Eq. (fle) with the albedo and phase function of the particle
    pre = air ? weight * rayleigh_phase(cosang) / r2 : A.albedo * weight * hg_phase(A.g, cosang) / r2;
    return true;
}

// Step (iv) in an air + aerosol mixture: the particle at collision s is air
// with probability beta_air / beta in the collision voxel, from the first
// word of Philox counter (pid_lo, pid_hi, s, 1).  Decided in FP64 for either
// transport precision, with beta = air + sig * aer rounded as in the
// library's copy of beta (no fused multiply-add).
template <typename Real>
__device__ __forceinline__ int mix_particle(const KArgs<Real>& A, const Photon<Real>& ph) {
    const int64_t k = (int64_t)ph.ix + (int64_t)A.G.nx * ph.iy + (int64_t)A.G.nxy * ph.iz;
    const double air = A.mix_air[k];
    const double tot = __dadd_rn(air, __dmul_rn(A.mix_sig, A.mix_aer[k]));
    const uint4 r = philox4x32_10(make_uint4((uint32_t)ph.pid, (uint32_t)(ph.pid >> 32), ph.s, 1u),
                                  make_uint2((uint32_t)A.seed, (uint32_t)(A.seed >> 32)));
    return uniform01<double>(r.x) < air / tot ? 1 : 0;
}

// Steps (v)-(vi) after collision s: returns -1 while the photon lives, else
// its fate (capped or ended by Russian roulette).
template <typename Real>
__device__ __forceinline__ int after_collision(const KArgs<Real>& A, Photon<Real>& ph) {
    if (ph.s >= A.max_events) return MC_FATE_CAP;
    const uint4 r = draw(A.seed, ph.pid, ph.s);
    if (!ph.air) ph.weight *= A.albedo;  // air: albedo 1
    if (ph.weight < A.rr) {
        if (uniform01<Real>(r.z) < ph.weight / A.rr) {
            ph.weight = A.rr;
        } else {
            return MC_FATE_RR;
        }
    }
    const Real omm = ph.air ? rayleigh_one_minus_mu(uniform01<Real>(r.x)) : hg_one_minus_mu(A.g, uniform01<Real>(r.x));
    scatter_direction(ph.wx, ph.wy, ph.wz, omm, uniform01<Real>(r.y));
    ph.taustar = -m_log((Real)1 - uniform01<Real>(r.w));
    return -1;
}

// ---------------------------------------------------------------------------
// Local-estimate jobs.

// LDS queue of one wavefront (structure of arrays, ring of QCAP entries).
template <typename Real, int MODE>
struct JobQueue {
    uint32_t vox[QCAP];  // start voxel packed as ix | iy << 11 | iz << 22
    Real fx[QCAP], fy[QCAP], fz[QCAP];
    Real vx[QCAP], vy[QCAP], vz[QCAP];
    Real r[QCAP], pre[QCAP];
    int32_t pix[QCAP];
    uint32_t evi[MODE == MODE_TAPE ? QCAP : 1];  // tape replay: the estimate's slot in its photon's row
};

// Sec. 3.2, Eq. (Lcupdate): a collision adds albedo I_s P(angle) to L_c of
// its voxel for every camera c, the angle between the incoming direction and
// the direction from the collision point to the camera centre.
//
// The wave's collisions (mask cm) are staged in its LDS queue and the
// (collision, camera) pairs are dealt to the lanes camera-fastest; lane l
// starts at pair l, i.e. at collision e0 = l / n_cams, camera c0 = l % n_cams,
// and steps by 64 pairs (e_step, c_step).  With L laid out [voxel][camera,
// padded to a multiple of 8] the atomics of one instruction fall on a few
// cache lines instead of 64, which the memory side combines.
template <typename Real, int MODE>
__device__ __forceinline__ void voxel_tally(const KArgs<Real>& A, JobQueue<Real, MODE>& Q, const Photon<Real>& ph,
                                            bool collided, unsigned long long cm, uint32_t e0, uint32_t c0,
                                            uint32_t e_step, uint32_t c_step, uint32_t& n_tally) {
    if (collided) {
        const uint32_t slot = lanes_below(cm);
        Q.vox[slot] = (uint32_t)ph.ix | ((uint32_t)ph.iy << 11) | ((uint32_t)ph.iz << 22);
        Q.fx[slot] = ph.fx;
        Q.fy[slot] = ph.fy;
        Q.fz[slot] = ph.fz;
        Q.vx[slot] = ph.wx;
        Q.vy[slot] = ph.wy;
        Q.vz[slot] = ph.wz;
        Q.pre[slot] = ph.weight;
    }
    __builtin_amdgcn_wave_barrier();
    const uint32_t n_e = (uint32_t)__popcll(cm);
    const uint32_t n_c = (uint32_t)A.n_cams;
    for (uint32_t e = e0, c = c0; e < n_e;) {
        const uint32_t v = Q.vox[e];
        const int ix = (int)(v & 2047u), iy = (int)((v >> 11) & 2047u), iz = (int)(v >> 22);
        const DevCam<Real>& cam = A.cams[c];
        // X_c - X from voxel-local parts (exact integer differences)
        const Real dx = ((Real)(cam.icx - ix) + (cam.fcx - Q.fx[e])) * A.G.dx;
        const Real dy = ((Real)(cam.icy - iy) + (cam.fcy - Q.fy[e])) * A.G.dy;
        const Real dz = ((Real)(cam.icz - iz) + (cam.fcz - Q.fz[e])) * A.G.dz;
        const Real r2 = dx * dx + dy * dy + dz * dz;
        if (r2 >= (Real)1e-12) {
            const Real cosang = (Q.vx[e] * dx + Q.vy[e] * dy + Q.vz[e] * dz) / m_sqrt(r2);
            const int64_t k = (int64_t)ix + (int64_t)A.G.nx * iy + (int64_t)A.G.nxy * iz;
            const double aw = (double)A.albedo * (double)Q.pre[e];
            unsafeAtomicAdd(A.Lc + k * A.lc_pitch + c, aw * (double)hg_phase(A.g, cosang));
            ++n_tally;
        }
        e += e_step;
        c += c_step;
        if (c >= n_c) {
            c -= n_c;
            ++e;
        }
    }
    // the next staging must not overtake this pass's reads
    __builtin_amdgcn_wave_barrier();
}

// Walk of a connection ray.  Its length is clipped at job start to where
// the ray leaves the domain, so that the walk ends at its length and keeps
// only the linear voxel index, not the voxel indices: the next crossing on
// axis a is t_a = r_a g_a as in the free-flight walk (r_a counted from the
// start voxel, t recomputed after every crossing), and a crossing that
// rounding put just before the clipped end (so that k left the grid) ends
// the walk too.
template <typename Real>
struct ConnWalk {
    int k, kx, ky, kz;
    int iz, izs;  // layer of the current voxel and its step on a z crossing
    Real sfx, sfy, sfz;
    Real rx, ry, rz;
    Real gx, gy, gz;
    Real tx, ty, tz;
    Real t;
};

// Start at voxel-local (i, f) along unit w; returns the parameter where the
// ray leaves the domain (inf when the walk cannot start: no usable
// direction component, or a non-finite fraction).
template <typename Real>
__device__ __forceinline__ Real conn_begin(ConnWalk<Real>& C, const DevGrid<Real>& G, int ix, int iy, int iz, Real fx,
                                           Real fy, Real fz, Real wx, Real wy, Real wz) {
    int sx, sy, sz;
    C.k = ix + G.nx * iy + G.nxy * iz;
    walk_axis(fx, wx, G.dx, sx, C.sfx, C.rx, C.gx, C.tx);
    walk_axis(fy, wy, G.dy, sy, C.sfy, C.ry, C.gy, C.ty);
    walk_axis(fz, wz, G.dz, sz, C.sfz, C.rz, C.gz, C.tz);
    C.kx = sx;
    C.ky = sy * G.nx;
    C.kz = sz * G.nxy;
    C.iz = iz;
    C.izs = sz;
    C.t = (Real)0;
    // the domain face on each axis lies (n - 1 - i) voxels beyond the first
    // face when moving up, i voxels beyond it when moving down
    const Real ex = sx > 0 ? ((Real)(G.nx - 1 - ix) + C.rx) * C.gx : (sx < 0 ? (C.rx - (Real)ix) * C.gx : (Real)INFINITY);
    const Real ey = sy > 0 ? ((Real)(G.ny - 1 - iy) + C.ry) * C.gy : (sy < 0 ? (C.ry - (Real)iy) * C.gy : (Real)INFINITY);
    const Real ez = sz > 0 ? ((Real)(G.nz - 1 - iz) + C.rz) * C.gz : (sz < 0 ? (C.rz - (Real)iz) * C.gz : (Real)INFINITY);
    const bool finite_f = fabs(fx) < (Real)4 && fabs(fy) < (Real)4 && fabs(fz) < (Real)4;
    if (!finite_f || (sx | sy | sz) == 0) return (Real)-1;
    return fmin(ex, fmin(ey, ez));
}

template <typename Real>
__device__ __forceinline__ Real conn_next(const ConnWalk<Real>& C, bool& cx, bool& cy, bool& cz) {
    cx = (C.tx <= C.ty) && (C.tx <= C.tz);
    cy = !cx && (C.ty <= C.tz);
    cz = !cx && !cy;
    return fmin(C.tx, fmin(C.ty, C.tz));
}

template <typename Real>
__device__ __forceinline__ void conn_cross(ConnWalk<Real>& C, Real tn, bool cx, bool cy, bool cz) {
    C.t = tn;
    C.k += (cx ? C.kx : 0) + (cy ? C.ky : 0) + (cz ? C.kz : 0);
    C.iz += cz ? C.izs : 0;
    C.rx += cx ? C.sfx : (Real)0;
    C.ry += cy ? C.sfy : (Real)0;
    C.rz += cz ? C.sfz : (Real)0;
    C.tx = C.rx * C.gx;
    C.ty = C.ry * C.gy;
    C.tz = C.rz * C.gz;
}

// One lane's connection ray in flight.  The optical depth of a voxel is
// added some steps after the walk left it, so that the fetch of its
// extinction has time to arrive, with fixed register roles (no copies):
//  * the walks without a second phase (render, tape) run in triples of steps
//    (job_step3<PH>) over a ring of three slots (b0, L0), (b1, L1), (b2, L2):
//    voxel m's extinction and length sit in slot m mod 3; step n adds the
//    term of voxel n - 2 and refills that slot with the length of voxel n
//    and the fetch for voxel n + 1, which is waited for two steps later;
//  * the gradient walk runs in pairs (job_step<PH>): in step PH, b[PH] is
//    the current voxel's extinction (in flight) and b[1-PH] the previous
//    voxel's, whose term b[1-PH] * lp is added and whose register then
//    receives the fetch for the next voxel, waited for one step later.
template <typename Real>
struct Job {
    ConnWalk<Real> W;
    Real r;        // length to the camera, then clipped to the domain
    Real b0, b1, b2;
    Real L0, L1, L2;  // lengths of the ring (triples)
    Real lp;          // length of the previous voxel (pairs)
    Real pre;      // albedo * I_s * P / r^2
    double tau;    // optical depth so far (FP64)
    double a;      // gradient weight of the second walk
    int pix;
    double gwp;    // gradient weight of the pixel (loaded when the ray starts, or 1)
    int phase;     // 1: optical depth, 2: gradient scatter
    uint32_t steps;
    uint32_t evi;  // tape replay of a mixture: slot of the estimate's collision in mix_rows
    // start of the ray, kept for the second walk of the gradient
    int i0x, i0y, i0z;
    Real f0x, f0y, f0z, vx, vy, vz;
};

// Step n (n mod 3 = PH) of a walk without a second phase; returns the
// wavefront's mask of the lanes whose ray ends at this step.  The whole wavefront steps together (no branch around
// the step, so that the compiler can count the fetches in flight and wait
// for the oldest only): a lane whose ray is done keeps stepping with its end
// clipped to where it stopped, i.e. with zero lengths and fetches of the
// shared zero word, which adds its two pending terms and nothing else.
// Exactly one axis crosses, so the index moves by one of kx, ky, kz; the
// occupancy bit of run c = k >> msh is bit c mod 32 of word k >> (msh + 5)
// (the bit-field extract reads the low 5 bits of its offset).
//
// AIRZ: the empty runs read the air column by layer (a mixture whose air
// depends on the height only), so the walk tracks its layer, and fetches
// with plain loads (the air column lies past the walk's buffer); otherwise
// the fetches go through the buffer.
template <typename Real, int PH, bool AIRZ>
__device__ __forceinline__ unsigned long long job_step3(const WalkCtx<Real>& C, const uint32_t* mask, uint32_t msh5,
                                                        Job<Real>& J, uint32_t& ld) {
    Real& bo = PH == 0 ? J.b1 : (PH == 1 ? J.b2 : J.b0);  // slot n - 2, i.e. n + 1
    Real& Lo = PH == 0 ? J.L1 : (PH == 1 ? J.L2 : J.L0);
    Real& Ln = PH == 0 ? J.L0 : (PH == 1 ? J.L1 : J.L2);  // slot n
    ConnWalk<Real>& W = J.W;
    // the axis that crosses first (x, then y on ties): the minimum is one of
    // the three values exactly
    const Real tn = fmin(W.tx, fmin(W.ty, W.tz));
    const bool cx = W.tx == tn;
    const bool cy = !cx && W.ty == tn;
    const bool last = tn >= J.r;
    const Real tend = last ? J.r : tn;
    J.tau += (double)bo * (double)Lo;
    Ln = tend - W.t;
    W.t = tend;
    const int kx = W.kx, ky = W.ky, kz = W.kz;  // values: a select of fields would select addresses
    W.k += cx ? kx : (cy ? ky : kz);
    if (AIRZ) W.iz += (!cx && !cy) ? W.izs : 0;
    W.rx += cx ? W.sfx : (Real)0;
    W.ry += cy ? W.sfy : (Real)0;
    W.rz += (!cx && !cy) ? W.sfz : (Real)0;
    W.tx = W.rx * W.gx;
    W.ty = W.ry * W.gy;
    W.tz = W.rz * W.gz;
    const bool past = (uint32_t)W.k >= C.n_vox;
    const bool done = last || past;
    J.r = done ? tend : J.r;
    // branch free: voxel 0 is a valid index to test when the ray is done
    const uint32_t kk = done ? 0u : (uint32_t)W.k;
    const bool occ = __builtin_amdgcn_ubfe(mask[kk >> msh5], kk >> C.msh, 1u) != 0u;
    ld = AIRZ ? (done ? C.n_vox : (occ ? kk : C.empty(W.iz))) : ((done || !occ) ? C.n_vox : kk);
    bo = C.template fetch<!AIRZ>(ld);
    // (a ballot of each test is that compare's own lane mask; one of their
    // OR would go through a vector register)
    return __builtin_amdgcn_ballot_w64(last) | __builtin_amdgcn_ballot_w64(past);
}

template <typename Real>
__device__ __forceinline__ void job_begin(const WalkCtx<Real>& C, const uint32_t* mask, Job<Real>& J) {
    const Real texit = conn_begin(J.W, C.G, J.i0x, J.i0y, J.i0z, J.f0x, J.f0y, J.f0z, J.vx, J.vy, J.vz);
    if (texit < (Real)0) {
        // cannot start: the first step ends the walk with zero length
        J.r = (Real)0;
        J.W.tx = J.W.ty = J.W.tz = (Real)0;
    } else {
        J.r = fmin(J.r, texit);
    }
    J.b0 = J.phase == 2 ? (Real)0 : C.load(mask, J.W.k, J.W.iz);
    J.b1 = J.b2 = (Real)0;
    J.L0 = J.L1 = J.L2 = J.lp = (Real)0;
    J.tau = 0.0;
    J.steps = 0;
}

// One voxel of the gradient's connection ray (step PH of a pair); returns
// true when the ray is done.
template <typename Real, int MODE, int TALLY, int PH>
__device__ __forceinline__ bool job_step(const KArgs<Real>& A, const uint32_t* mask, double* lds_grad, Job<Real>& J) {
    Real& prev = PH == 0 ? J.b1 : J.b0;
    bool cx, cy, cz;
    const Real tn = conn_next(J.W, cx, cy, cz);
    const bool last = tn >= J.r;
    const Real tend = last ? J.r : tn;
    const Real l = tend - J.W.t;
    if (MODE == MODE_GRAD && J.phase == 2) {
        // second walk of the gradient: only the deposit.  A crossing within
        // a few ulps of the clipped end is taken as the end: past a side face
        // of the domain the linear index would wrap into another voxel, which
        // would receive the ray's last sliver
        const Real near_end = J.r * (Real)(sizeof(Real) == 4 ? 1.0 - 0x1p-18 : 1.0 - 0x1p-44);
        const bool end = last || tn >= near_end;
        grad_add<Real, TALLY>(A, lds_grad, J.W.k, -J.a * (double)((end ? J.r : tn) - J.W.t));
        conn_cross(J.W, tn, cx, cy, cz);
        return end || (uint32_t)J.W.k >= (uint32_t)A.n_vox;
    }
    J.tau += (double)prev * (double)J.lp;
    J.lp = l;
    ++J.steps;
    conn_cross(J.W, tn, cx, cy, cz);
    const bool done = last || (uint32_t)J.W.k >= (uint32_t)A.n_vox;
    // the next fetch is issued unconditionally (the shared zero word when the
    // ray is done or enters an empty run).  When the ray is done,
    // the last voxel's term cur * lp is left to job_finish, as
    // (b0 + b1) * lp with the other register zero, so that no step waits for
    // a fetch it has just issued.
    // (branch free: the job phase always has the LDS mask, and voxel 0 is a
    // valid index to test when the ray is done)
    const int kk = done ? 0 : J.W.k;
    const bool none = (int)done | (int)!occupied(A, mask, kk);
    prev = A.beta_le[none ? (uint32_t)A.n_vox : (uint32_t)kk];
    return done;
}

// Tally of a finished ray.  For the gradient, a finished first walk with a
// non-zero weight starts the second walk (returns true: the lane stays busy);
// for the tape, such a ray is marked for the tape (rec) instead.
template <typename Real, typename W, int MODE, int TALLY>
__device__ __forceinline__ bool job_finish(const KArgs<Real>& A, const WalkCtx<W>& C, const uint32_t* mask,
                                           double* lds_grad, Job<W>& J, uint64_t& vconn, bool& rec) {
    if (MODE == MODE_GRAD && J.phase == 2) return false;
    if (MODE == MODE_GRAD) {
        vconn += J.steps;
        J.tau += ((double)J.b0 + (double)J.b1) * (double)J.lp;  // the last voxel
    } else {
        // the two voxels still pending (the other slots hold a zero fetch or
        // a zero length)
        J.tau += (double)J.b0 * (double)J.L0;
        J.tau += (double)J.b1 * (double)J.L1;
        J.tau += (double)J.b2 * (double)J.L2;
    }
    // (the tape replay of a mixture queues an air collision's estimates with
    // pre negated, the mark its ray record carries)
    const W pre = MODE == MODE_TAPE ? (W)fabs(J.pre) : J.pre;
    // the transmittance in the walk's precision (mixed precision: FP32, about
    // 1e-7 relative; an FP64 exp per estimate cost the mixed render 4%, its
    // constants held in registers the photon phase then spills)
    const double tr = (double)m_exp((W)(-J.tau));
    const double ce = (double)pre * tr;
    if (MODE == MODE_RENDER || MODE == MODE_RTAPE) {
        tally_f64<TALLY>(A.img, A.img32, J.pix, ce);
        if (A.img_m2) unsafeAtomicAdd(A.img_m2 + J.pix, ce * ce);
        if (MODE == MODE_RTAPE) {
            J.a = ce;
            rec = ce != 0.0;
        }
        return false;
    } else if (MODE == MODE_TAPE) {
        J.a = J.gwp * ce;
        // full gradient of a mixture: a = gw C summed per collision
        if (A.mix_rows && J.a != 0.0) unsafeAtomicAdd(A.mix_rows + J.evi, J.a);
        if (A.mix_aer) J.a = A.mix_sig * J.a;  // the aerosol field's derivative of beta
        rec = J.a != 0.0;
        return false;
    } else {
        const double a = A.gw[J.pix] * ce;
        if (a == 0.0) return false;
        const int ke = J.i0x + A.G.nx * J.i0y + A.G.nxy * J.i0z;
        grad_add<Real, TALLY>(A, lds_grad, ke, a / (double)A.beta[ke]);
        J.a = a;
        J.phase = 2;
        job_begin(C, mask, J);
        return true;
    }
}

// The rays marked by job_finish go to the wavefront's slice of the ray tape,
// in consecutive slots (one coalesced store per finishing batch; a wait on
// a later load also waits for these stores, so they are made once per
// batch, not per tile).  w_used counts the wavefront's rays, also past the
// end of its slice (the host then replays the chunk smaller).
template <typename Real, typename W>
__device__ __forceinline__ void tape_write(const KArgs<Real>& A, const Job<W>& J, bool rec, uint32_t& w_used,
                                           uint32_t w_first) {
    const unsigned long long m = __ballot(rec);
    if (!m) return;
    if (rec) {
        const uint32_t pos = w_used + lanes_below(m);
        if (pos < A.tp.rw) {
            TapeRec<Real> R;
            R.vox = (uint32_t)J.i0x | ((uint32_t)J.i0y << 11) | ((uint32_t)J.i0z << 22);
            R.id = (uint32_t)J.pix;
            R.fx = J.f0x;
            R.fy = J.f0y;
            R.fz = J.f0z;
            R.a = (Real)J.a;
            R.ab = J.pre < (Real)0 ? (Real)0 : (Real)1;
            A.tp.rec[w_first + pos] = R;
        }
    }
    w_used += (uint32_t)__popcll(m);
}

// Job phase of one wavefront.  Not final: return once fewer jobs are queued
// or in flight than there are lanes.  Final: run until everything is done.
// CAP: every step of the walks stores its loaded index for the gather
// capture (wstep counts the wavefront's steps).
template <typename Real, typename W, int MODE, int TALLY, bool AIRZ, bool CAP = false>
__device__ __forceinline__ void drain(const KArgs<Real>& A, const WalkCtx<W>& C, const uint32_t* mask,
                                      double* lds_grad, JobQueue<W, MODE>& Q, uint32_t& qhead, uint32_t qtail,
                                      Job<W>& J, bool& busy, bool& fin, bool final_pass, uint64_t& vconn,
                                      uint64_t& vconn_w, uint32_t& w_used, uint32_t w_first, uint32_t& wstep,
                                      uint32_t wave_id) {
    for (;;) {
        bool rec = false;
        if (fin) {
            fin = false;
            busy = job_finish<Real, W, MODE, TALLY>(A, C, mask, lds_grad, J, vconn, rec);
        }
        if constexpr (MODE == MODE_TAPE || MODE == MODE_RTAPE) tape_write(A, J, rec, w_used, w_first);
        const uint32_t count = qtail - qhead;
        const uint32_t nbusy = (uint32_t)__popcll(__ballot(busy));
        if (final_pass ? (count + nbusy == 0) : (count + nbusy < (uint32_t)WAVE)) break;
        if (count > 0) {
            const unsigned long long idle = __ballot(!busy);
            const uint32_t take = min((uint32_t)__popcll(idle), count);
            if (!busy) {
                const uint32_t rank = lanes_below(idle);
                if (rank < take) {
                    const uint32_t slot = (qhead + rank) & (QCAP - 1);
                    const uint32_t v = Q.vox[slot];
                    J.i0x = (int)(v & 2047u);
                    J.i0y = (int)((v >> 11) & 2047u);
                    J.i0z = (int)(v >> 22);
                    J.f0x = Q.fx[slot];
                    J.f0y = Q.fy[slot];
                    J.f0z = Q.fz[slot];
                    J.vx = Q.vx[slot];
                    J.vy = Q.vy[slot];
                    J.vz = Q.vz[slot];
                    J.r = Q.r[slot];
                    J.pre = Q.pre[slot];
                    J.pix = Q.pix[slot];
                    if (MODE == MODE_TAPE) {
                        // the weight of the pixel, needed when the ray
                        // finishes, unless the binning pass applies it
                        // (scale_gw): a gather that misses L2 would hold up
                        // the walk's first loads (vector loads complete in
                        // order)
                        J.gwp = A.tp.scale_gw ? 1.0 : A.gw[J.pix];
                        if (A.mix_rows) J.evi = Q.evi[slot];
                    }
                    J.phase = 1;
                    job_begin(C, mask, J);
                    busy = true;
                }
            }
            qhead += take;
        }
        // walk until a quarter of the lanes are idle (all, if nothing is
        // queued), in pairs (gradient) or triples of steps (a job always
        // starts with step 0)
        const uint32_t keep = (qtail - qhead) > 0 ? (uint32_t)WAVE - REFILL_IDLE : 0u;
        if constexpr (MODE == MODE_GRAD) {
            while ((uint32_t)__popcll(__ballot(busy)) > keep) {
                if (busy) {
                    const bool d = job_step<Real, MODE, TALLY, 0>(A, mask, lds_grad, J);
                    busy = !d;
                    fin = d;
                }
                if (busy) {
                    const bool d = job_step<Real, MODE, TALLY, 1>(A, mask, lds_grad, J);
                    busy = !d;
                    fin = d;
                }
            }
        } else {
            // voxel steps are counted per wavefront: the busy lanes of each
            // step.  The busy and finished lanes are kept as wavefront masks
            // (scalar registers), updated from each step's mask of ended rays
            const uint32_t msh5 = (uint32_t)C.msh + 5u;
            unsigned long long bm = __ballot(busy), fm = __ballot(fin);
            auto capture = [&](uint32_t ld) {
                if constexpr (CAP) {
                    const uint32_t j = wstep - A.cap_first;
                    if (j < A.cap_steps) A.capture[((size_t)wave_id * A.cap_steps + j) * WAVE + __lane_id()] = ld;
                    ++wstep;
                }
            };
            for (;;) {
                uint32_t ld0, ld1, ld2;
                const uint32_t n0 = (uint32_t)__popcll(bm);
                if (n0 <= keep) break;
                const unsigned long long m0 = job_step3<W, 0, AIRZ>(C, mask, msh5, J, ld0);
                capture(ld0);
                fm |= bm & m0;
                bm &= ~m0;
                const uint32_t n1 = (uint32_t)__popcll(bm);
                const unsigned long long m1 = job_step3<W, 1, AIRZ>(C, mask, msh5, J, ld1);
                capture(ld1);
                fm |= bm & m1;
                bm &= ~m1;
                const uint32_t n2 = (uint32_t)__popcll(bm);
                const unsigned long long m2 = job_step3<W, 2, AIRZ>(C, mask, msh5, J, ld2);
                capture(ld2);
                fm |= bm & m2;
                bm &= ~m2;
                vconn_w += n0 + n1 + n2;
            }
            busy = ((bm >> __lane_id()) & 1ull) != 0ull;
            fin = ((fm >> __lane_id()) & 1ull) != 0ull;
        }
    }
}

// Wavefronts per SIMD the compiler must leave room for: 4 (at most 128
// VGPRs) for the FP32 kernels and the mixed-precision render, which are
// latency bound and gain more from a fourth wavefront than they lose to the
// tighter register budget (the mixed render then spills some of its FP64
// photon state in the photon phase and is still 2% faster than with three);
// the FP64 kernels keep their registers.
template <typename Real, int MODE, bool W32 = false>
struct RenderWaves {
    static constexpr int value = (sizeof(Real) == 4 && MODE != MODE_TRACE && MODE != MODE_BMC) || W32 ? 4 : 1;
};

// Threads per block: 512 for the gradient, whose privatised copy of the
// gradient (up to 64 KB of LDS per block) is then shared by 8 wavefronts, so
// that the copies do not limit the wavefronts per CU; 256 otherwise.
template <int MODE>
struct RenderThreads {
    static constexpr int value = MODE == MODE_GRAD ? 512 : 256;
};

// Dynamic LDS of k_render: the occupancy bitmask (mask_words), then, when
// the gradient is privatised, one double per voxel.
//
// W32 (mixed precision, Real = double): the photons fly, collide and
// scatter in FP64 exactly as in the FP64 kernel, while the connection rays
// walk a float copy of beta in FP32 (optical depths still summed in FP64).
//
// CAP (FP32 render only): the gather capture, a diagnostic.
template <typename Real, int MODE, int TALLY, bool AIRZ = false, bool W32 = false, bool CAP = false>
__global__ void __launch_bounds__((RenderThreads<MODE>::value), (RenderWaves<Real, MODE, W32>::value))
    k_render(KArgs<Real> A) {
    using W = typename WalkPrec<Real, W32>::type;
    constexpr int NT = RenderThreads<MODE>::value;
    constexpr int NW = NT / WAVE;
    __shared__ JobQueue<W, MODE> s_q[NW];
    __shared__ unsigned long long s_st[ST_N];
    extern __shared__ uint32_t s_dyn[];
    uint32_t* s_mask = s_dyn;
    double* lds_grad = nullptr;
    if (MODE == MODE_GRAD && A.grad_lds) {
        lds_grad = reinterpret_cast<double*>(s_dyn + ((A.mask_words + 1) & ~1));
        for (int64_t i = threadIdx.x; i < A.n_vox; i += NT) lds_grad[i] = 0.0;
    }
    if (threadIdx.x < ST_N) s_st[threadIdx.x] = 0ull;
    for (int i = threadIdx.x; i < A.mask_words; i += NT) s_mask[i] = A.mask[i];
    __syncthreads();
    const uint32_t* mask = s_mask;
    JobQueue<W, MODE>& Q = s_q[threadIdx.x / WAVE];
    const WalkCtx<W> C = walk_ctx<Real, W32>(A);

    Photon<Real> ph;
    Job<W> J{};
    bool alive = false, exhausted = false, busy = false, fin = false;
    uint64_t pool_next = 0, pool_end = 0;
    uint32_t qhead = 0, qtail = 0;
    uint32_t n_ev = 0, n_le = 0;
    uint32_t kloc = 0;  // the lane's photon within the launch (tape replay)
    uint64_t vfree = 0, vconn = 0;
    uint64_t vconn_w = 0;  // counted per wavefront (the same in every lane)
    const uint32_t wave_id = blockIdx.x * NW + threadIdx.x / WAVE;
    const uint32_t w_first = MODE == MODE_TAPE || MODE == MODE_RTAPE ? wave_id * A.tp.rw : 0u;
    uint32_t w_used = 0;
    uint32_t wstep = 0;  // the wavefront's walk steps (gather capture)
    // voxel tally: this lane's first (collision, camera) pair and the step
    const uint32_t n_c = A.n_cams > 0 ? (uint32_t)A.n_cams : 1u;
    const uint32_t v_e0 = __lane_id() / n_c, v_c0 = __lane_id() % n_c;
    const uint32_t v_estep = (uint32_t)WAVE / n_c, v_cstep = (uint32_t)WAVE % n_c;

    for (;;) {
        const unsigned long long need = __ballot(!alive && !exhausted);
        if (need) {
            const uint64_t k = wave_fetch(A.work, A.fetch_block, need, pool_next, pool_end);
            if (!alive && !exhausted) {
                if (k < A.n_photons) {
                    launch_photon(A, A.pid0 + k, ph);
                    kloc = (uint32_t)k;
                    alive = true;
                } else {
                    exhausted = true;
                }
            }
        }
        if (__ballot(alive) == 0ull) break;
        bool collided = false;
        if (alive) {
            const int left = free_flight(A, mask, ph, vfree, FLIGHT_BUDGET);
            if (left == FLIGHT_GOES_ON) {
                // still flying: continues at the next photon phase
            } else if (left) {
                atomicAdd(&s_st[ST_TOP + left - 1], 1ull);
                alive = false;
            } else {
                collided = true;
                ph.s += 1;
                ++n_ev;
                if (A.mix_air) ph.air = mix_particle(A, ph);
            }
        }
        if constexpr (MODE == MODE_VOXEL) {
            const unsigned long long cm = __ballot(collided);
            if (cm && A.n_cams > 0) voxel_tally<Real, MODE>(A, Q, ph, collided, cm, v_e0, v_c0, v_estep, v_cstep, n_le);
        } else if (__ballot(collided)) {
            // frozen-event render: the estimate scaled by beta_le / beta at the collision
            Real fr = (Real)1;
            if (A.frozen && collided) {
                const int64_t k = (int64_t)ph.ix + (int64_t)A.G.nx * ph.iy + (int64_t)A.G.nxy * ph.iz;
                fr = (Real)((double)A.beta_le[k] / (double)A.beta[k]);
            }
            for (int c = 0; c < A.n_cams; ++c) {
                const DevCam<Real>& cam = A.cams[c];
                int64_t pix = 0;
                int lp = 0;
                Real vx = 0, vy = 0, vz = 0, r = 0, pre = 0;
                const bool vis = collided && le_geometry(A, cam, ph.ix, ph.iy, ph.iz, ph.fx, ph.fy, ph.fz, ph.wx,
                                                         ph.wy, ph.wz, ph.weight, ph.air, pix, lp, vx, vy, vz, r, pre);
                const unsigned long long m = __ballot(vis);
                if (vis) {
                    const uint32_t slot = (qtail + lanes_below(m)) & (QCAP - 1);
                    Q.vox[slot] = (uint32_t)ph.ix | ((uint32_t)ph.iy << 11) | ((uint32_t)ph.iz << 22);
                    Q.fx[slot] = ph.fx;
                    Q.fy[slot] = ph.fy;
                    Q.fz[slot] = ph.fz;
                    Q.vx[slot] = vx;
                    Q.vy[slot] = vy;
                    Q.vz[slot] = vz;
                    Q.r[slot] = r;
                    Q.pre[slot] = MODE == MODE_TAPE && ph.air ? -pre : (A.frozen ? pre * fr : pre);
                    Q.pix[slot] = (int32_t)pix;
                    if (MODE == MODE_TAPE && A.mix_rows)
                        Q.evi[slot] = kloc * (A.mix_evcap + 1u) + min(ph.s - 1u, A.mix_evcap);
                    ++n_le;
                }
                qtail += (uint32_t)__popcll(m);
                if (qtail - qhead > QCAP - (uint32_t)WAVE)
                    drain<Real, W, MODE, TALLY, AIRZ, CAP>(A, C, mask, lds_grad, Q, qhead, qtail, J, busy, fin, false,
                                                           vconn, vconn_w, w_used, w_first, wstep, wave_id);
            }
        }
        if (collided) {
            const int fate = after_collision(A, ph);
            if (fate >= 0) {
                atomicAdd(&s_st[fate == MC_FATE_CAP ? ST_CAP : ST_RR], 1ull);
                alive = false;
            }
        }
        drain<Real, W, MODE, TALLY, AIRZ, CAP>(A, C, mask, lds_grad, Q, qhead, qtail, J, busy, fin, false, vconn,
                                               vconn_w, w_used, w_first, wstep, wave_id);
    }
    drain<Real, W, MODE, TALLY, AIRZ, CAP>(A, C, mask, lds_grad, Q, qhead, qtail, J, busy, fin, true, vconn, vconn_w,
                                           w_used, w_first, wstep, wave_id);
    if (CAP && __lane_id() == 0) A.capture_steps[wave_id] = wstep;

    if ((MODE == MODE_TAPE || MODE == MODE_RTAPE) && __lane_id() == 0) {
        A.tp.wave_count[wave_id] = w_used;
        if (w_used > A.tp.rw) A.tp.overflow[0] = 1u;
    }
    if (n_ev) atomicAdd(&s_st[ST_EVENTS], (unsigned long long)n_ev);
    if (n_le) atomicAdd(&s_st[ST_LE], (unsigned long long)n_le);
    if (vfree) atomicAdd(&s_st[ST_VFREE], (unsigned long long)vfree);
    if (__lane_id() == 0) vconn += vconn_w;
    if (vconn) atomicAdd(&s_st[ST_VCONN], (unsigned long long)vconn);
    __syncthreads();
    if (threadIdx.x < ST_N && s_st[threadIdx.x]) atomicAdd(&A.stats[threadIdx.x], s_st[threadIdx.x]);
    if (lds_grad) {
        for (int64_t i = threadIdx.x; i < A.n_vox; i += NT) {
            const double v = lds_grad[i];
            if (v != 0.0) tally_f64<TALLY>(A.grad, A.grad32, i, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Binning of the ray tape by gradient tile.

// Ray of a tape record going to camera c: start voxel, unit direction to the
// camera and length, recomputed as the local estimate formed them.  False
// for a record outside the grid or the camera table.
template <typename Real>
__device__ __forceinline__ bool tape_ray(const KArgs<Real>& A, const TapeRec<Real>& R, uint32_t c, int& ix, int& iy,
                                         int& iz, Real& vx, Real& vy, Real& vz, Real& r) {
    ix = (int)(R.vox & 2047u);
    iy = (int)((R.vox >> 11) & 2047u);
    iz = (int)(R.vox >> 22);
    if (ix >= A.G.nx || iy >= A.G.ny || iz >= A.G.nz || c >= (uint32_t)A.n_cams) return false;
    const DevCam<Real>& cam = A.cams[c];
    const Real dx = ((Real)(ix - cam.icx) + (R.fx - cam.fcx)) * A.G.dx;
    const Real dy = ((Real)(iy - cam.icy) + (R.fy - cam.fcy)) * A.G.dy;
    const Real dz = ((Real)(iz - cam.icz) + (R.fz - cam.fcz)) * A.G.dz;
    r = m_sqrt(dx * dx + dy * dy + dz * dz);
    const Real ir = (Real)1 / r;
    vx = -dx * ir;
    vy = -dy * ir;
    vz = -dz * ir;
    return true;
}

// Calls f(tile) for every tile the ray crosses, in order (a walk over the
// grid of tiles; a ray without a usable direction only has its start tile).
template <typename Real, typename F>
__device__ __forceinline__ void for_each_tile(const Tape<Real>& P, const TapeRec<Real>& R, int ix, int iy, int iz,
                                              Real vx, Real vy, Real vz, Real r, F&& f) {
    WalkRegs<Real> W;
    const int tix = ix >> P.shx, tiy = iy >> P.shy, tiz = iz >> P.shz;
    const Real ftx = ((Real)(ix & ((1 << P.shx) - 1)) + R.fx) * P.itx;
    const Real fty = ((Real)(iy & ((1 << P.shy) - 1)) + R.fy) * P.ity;
    const Real ftz = ((Real)(iz & ((1 << P.shz) - 1)) + R.fz) * P.itz;
    if (!walk_begin(W, P.T, tix, tiy, tiz, ftx, fty, ftz, vx, vy, vz)) {
        f(tix + P.T.nx * tiy + P.T.nxy * tiz);
        return;
    }
    for (;;) {
        f(W.k);
        bool cx, cy, cz;
        const Real tn = walk_next(W, cx, cy, cz);
        if (tn >= r || walk_cross(W, P.T, tn, cx, cy, cz)) return;
    }
}

// Camera of global pixel p: the last camera whose first pixel is <= p
// (binary search over the cameras' first pixels: in LDS for the first
// BIN_LDS_CAMS cameras, else in the device table).
template <typename Real>
__device__ __forceinline__ uint32_t camera_of(const KArgs<Real>& A, const int32_t* s_off, uint32_t p) {
    int lo = 0, hi = A.n_cams - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int32_t off = mid < BIN_LDS_CAMS ? s_off[mid] : A.cams[mid].pix_off;
        if ((uint32_t)off <= p) lo = mid;
        else hi = mid - 1;
    }
    return (uint32_t)lo;
}

// Every ray of the block's part of its wavefront slice (part
// blockIdx.x % split of slice w0 + blockIdx.x / split): f(record with its
// weight and camera index, start voxel, direction, length).  A tape of local
// estimates (scale_gw) takes the weight gw[pixel] * a here; rays of zero
// weight are skipped.
template <typename Real, typename F>
__device__ __forceinline__ void for_each_block_ray(const KArgs<Real>& A, const int32_t* s_off, F&& f) {
    const Tape<Real>& P = A.tp;
    const uint32_t split = (uint32_t)P.split;
    const size_t w = (size_t)P.w0 + blockIdx.x / split;
    const uint64_t n = min(P.wave_count[w], P.rw), part = blockIdx.x % split;
    const uint32_t j0 = (uint32_t)(n * part / split), j1 = (uint32_t)(n * (part + 1) / split);
    for (uint32_t j = j0 + threadIdx.x; j < j1; j += BLOCK) {
        TapeRec<Real> R = P.rec[w * P.rw + j];
        if (P.scale_gw) R.a = (Real)((R.id < (uint32_t)A.n_pix ? A.gw[R.id] : 0.0) * (double)R.a);
        if (R.a == (Real)0) continue;
        R.id = camera_of(A, s_off, R.id);
        int ix, iy, iz;
        Real vx, vy, vz, r;
        if (tape_ray(A, R, R.id, ix, iy, iz, vx, vy, vz, r)) f(R, ix, iy, iz, vx, vy, vz, r);
    }
}

// Count pass (scatter = 0): for every tile t, the records of the block's
// rays in t go to slice[t][block] and are added to tile_count[t].
// Scatter pass (scatter = 1), after the scan: every ray, with its camera in
// place of its pixel, is copied into the bin of every tile in [t_lo, t_hi)
// it crosses, at the block's slots from slice[t][block] on.  Both passes run
// the same code, so they find the same tiles; should they ever disagree, a
// block only fills its own slots (extra records are dropped, unfilled slots
// get empty records with a = 0), so every bin slot holds valid data.
//
// Dynamic LDS: the first pixels of the cameras (bin_cams words), then one
// counter per tile of the pass, and for the scatter two more per tile.
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_bin(KArgs<Real> A, int scatter) {
    extern __shared__ uint32_t s_bin[];
    const Tape<Real>& P = A.tp;
    const int lo = scatter ? P.t_lo : 0, hi = scatter ? P.t_hi : P.n_tiles;
    const int n_off = min(A.n_cams, BIN_LDS_CAMS);
    const int b = blockIdx.x;
    int32_t* s_off = reinterpret_cast<int32_t*>(s_bin);
    uint32_t* s_cnt = s_bin + n_off;
    uint32_t* s_base = s_cnt + (hi - lo);
    uint32_t* s_lim = s_base + (hi - lo);
    for (int i = threadIdx.x; i < hi - lo; i += BLOCK) {
        s_cnt[i] = 0u;
        if (scatter) {
            const size_t row = (size_t)(lo + i) * P.n_slices;
            const uint32_t first = P.slice[row + b];
            const uint32_t next = b + 1 < P.n_slices ? P.slice[row + b + 1] : P.tile_end[lo + i];
            s_base[i] = first;
            s_lim[i] = next > first ? next - first : 0u;
        }
    }
    for (int i = threadIdx.x; i < n_off; i += BLOCK) s_off[i] = A.cams[i].pix_off;
    __syncthreads();
    for_each_block_ray(A, s_off, [&](const TapeRec<Real>& R0, int ix, int iy, int iz, Real vx, Real vy, Real vz, Real r) {
        TapeRec<Real> R = R0;
        if (scatter) {
            const int64_t k = ix + A.G.nx * iy + A.G.nxy * iz;
            if (A.mix_aer)  // the collision's score term: aerosol only, over the aerosol extinction
                R.ab = R.ab != (Real)0 ? (Real)((double)R.a / __dmul_rn(A.mix_sig, A.mix_aer[k])) : (Real)0;
            else
                R.ab = (Real)((double)R.a / (double)A.beta[k]);
        }
        for_each_tile(P, R, ix, iy, iz, vx, vy, vz, r, [&](int t) {
            if (t >= lo && t < hi) {
                const uint32_t p = atomicAdd(&s_cnt[t - lo], 1u);
                if (scatter && p < s_lim[t - lo]) P.brec[s_base[t - lo] + p] = R;
            }
        });
    });
    __syncthreads();
    if (!scatter) {
        for (int i = threadIdx.x; i < hi - lo; i += BLOCK) {
            const uint32_t n = s_cnt[i];
            P.slice[(size_t)(lo + i) * P.n_slices + b] = n;
            if (n) atomicAdd(&P.tile_count[lo + i], n);
        }
        return;
    }
    TapeRec<Real> E;
    E.vox = 0u;
    E.id = 0u;
    E.fx = E.fy = E.fz = E.a = E.ab = (Real)0;
    for (int i = 0; i < hi - lo; ++i)
        for (uint32_t p = s_cnt[i] + threadIdx.x; p < s_lim[i]; p += BLOCK) P.brec[s_base[i] + p] = E;
}

// Scan of the count pass: for each tile t of [t_lo, t_hi) (one block per
// tile), slice[t][b] becomes bin_start[t] + the records of slices 0..b-1.
template <typename Real>
__global__ void __launch_bounds__(SCAN_BLOCK) k_bin_scan(KArgs<Real> A) {
    __shared__ uint32_t s_sum[SCAN_BLOCK];
    const Tape<Real>& P = A.tp;
    const int t = P.t_lo + blockIdx.x;
    const int n = P.n_slices;
    uint32_t* row = P.slice + (size_t)t * n;
    const int per = (n + SCAN_BLOCK - 1) / SCAN_BLOCK;
    const int i0 = min(n, (int)threadIdx.x * per), i1 = min(n, i0 + per);
    uint32_t sum = 0u;
    for (int i = i0; i < i1; ++i) sum += row[i];
    s_sum[threadIdx.x] = sum;
    __syncthreads();
    // inclusive scan of the per-thread sums (Hillis-Steele)
    for (int d = 1; d < SCAN_BLOCK; d <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)d ? s_sum[threadIdx.x - d] : 0u;
        __syncthreads();
        s_sum[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = P.bin_start[t] + (threadIdx.x ? s_sum[threadIdx.x - 1] : 0u);
    for (int i = i0; i < i1; ++i) {
        const uint32_t c = row[i];
        row[i] = run;
        run += c;
    }
}

// ---------------------------------------------------------------------------
// Gradient deposit of one tile: the block accumulates in LDS, for the binned
// records [lo, hi) of its tile, -a l(m) along every recorded ray inside the
// tile and a / beta(k_e) for the rays that start in it, then adds the tile
// to the gradient (one device atomic per touched voxel).

// Walk of a deposit inside one tile.  The ray is clipped to the tile box
// beforehand, so the walk ends at its length and needs no voxel indices:
// only the linear index k (the LDS index) and the next crossing on each axis,
// advanced by the per-voxel increment dt = d / |w| (in FP32 the error of the
// crossings grows by an ulp per step; the error of a segment stays far
// below the Monte Carlo noise).  Axes the ray does not move along have
// dt = inf and are never chosen.
template <typename Real>
struct DepWalk {
    int k, kx, ky, kz;  // LDS byte offset of the voxel, and its step on each axis
    Real tx, ty, tz;
    Real dtx, dty, dtz;
    Real t, len;
};

// Camera centre in voxel units (integer and fraction), as the deposit keeps
// it in LDS.
template <typename Real>
struct alignas(16) CamCentre {
    int ix, iy, iz;
    Real fx, fy, fz;
};

// Start the deposit of binned record R: a / beta(k_e) if the ray starts in
// the tile, then the walk of the part of the ray inside the tile (false
// when the record is empty or that part has no length).  Straight-line code
// with selects: the lanes that start a record do so together, and branches
// would cost more in mask handling than the arithmetic they skip.
template <typename Real, bool CAMS_LDS>
__device__ __forceinline__ bool deposit_begin(const KArgs<Real>& A, const DevGrid<Real>& L, int px, int pxy, int b0x,
                                              int b0y, int b0z, const CamCentre<Real>* s_cam, const TapeRec<Real>& R,
                                              double* s_g, DepWalk<Real>& D, double& a) {
    a = (double)R.a;
    const int i0x = (int)(R.vox & 2047u), i0y = (int)((R.vox >> 11) & 2047u), i0z = (int)(R.vox >> 22);
    // (bitwise operators: no short-circuit branches)
    bool ok = (R.a != (Real)0) & (i0x < A.G.nx) & (i0y < A.G.ny) & (i0z < A.G.nz) & (R.id < (uint32_t)A.n_cams);
    const uint32_t c = ok ? R.id : 0u;  // keeps the camera read in bounds
    // all cameras in LDS, or all read from global memory: one kind of load
    // (a choice per lane would become a generic-address load)
    CamCentre<Real> cc;
    if (CAMS_LDS) {
        cc = s_cam[c];
    } else {
        const DevCam<Real>& cam = A.cams[c];
        cc.ix = cam.icx;
        cc.iy = cam.icy;
        cc.iz = cam.icz;
        cc.fx = cam.fcx;
        cc.fy = cam.fcy;
        cc.fz = cam.fcz;
    }
    // direction and length to the camera, as the local estimate formed them
    const Real dx = ((Real)(i0x - cc.ix) + (R.fx - cc.fx)) * A.G.dx;
    const Real dy = ((Real)(i0y - cc.iy) + (R.fy - cc.fy)) * A.G.dy;
    const Real dz = ((Real)(i0z - cc.iz) + (R.fz - cc.fz)) * A.G.dz;
    const Real r = m_sqrt_fast(dx * dx + dy * dy + dz * dz);
    const Real ir = m_rcp(r);
    const Real vx = -dx * ir, vy = -dy * ir, vz = -dz * ir;
    const int jx = i0x - b0x, jy = i0y - b0y, jz = i0z - b0z;
    if (ok && (unsigned)jx < (unsigned)L.nx && (unsigned)jy < (unsigned)L.ny && (unsigned)jz < (unsigned)L.nz)
        atomicAdd(s_g + (jx + px * jy + pxy * jz), (double)R.ab);
    // clip [0, r] to the tile box; o = start in tile-local voxel units,
    // w = km per voxel along each axis.  An axis the ray does not move along
    // (|v| <= tiny) does not clip; the ray must then lie within the tile's
    // slab of that axis, and a ray in the plane of a face belongs to the
    // tile above it.
    const Real tiny = sizeof(Real) == 4 ? (Real)1e-20f : (Real)1e-200;
    const Real o[3] = {(Real)jx + R.fx, (Real)jy + R.fy, (Real)jz + R.fz};
    const Real v[3] = {vx, vy, vz};
    const Real d[3] = {A.G.dx, A.G.dy, A.G.dz};
    const Real id[3] = {A.G.idx, A.G.idy, A.G.idz};
    const int e[3] = {L.nx, L.ny, L.nz};
    // LDS byte offsets: the walk adds them to the address it deposits at
    const int stride[3] = {(int)sizeof(double), (int)sizeof(double) * px, (int)sizeof(double) * pxy};
    bool mov[3];
    Real w[3];
    Real t0 = (Real)0, t1 = r;
    for (int ax = 0; ax < 3; ++ax) {
        mov[ax] = fabs(v[ax]) > tiny;
        w[ax] = d[ax] * m_rcp(mov[ax] ? v[ax] : (Real)1);
        const Real ta = ((Real)0 - o[ax]) * w[ax], tb = ((Real)e[ax] - o[ax]) * w[ax];
        t0 = mov[ax] ? fmax(t0, fmin(ta, tb)) : t0;
        t1 = mov[ax] ? fmin(t1, fmax(ta, tb)) : t1;
        ok &= mov[ax] | ((o[ax] >= (Real)0) & (o[ax] < (Real)e[ax]));
    }
    ok &= t1 > t0;
    int ks[3];
    Real tn[3], dt[3];
    D.k = 0;
    for (int ax = 0; ax < 3; ++ax) {
        // entry voxel and fraction; the first crossing; the increment
        const Real p = o[ax] + t0 * v[ax] * id[ax];
        const Real fl = fmin(fmax(m_floor(p), (Real)0), (Real)(e[ax] - 1));
        const Real fr = fmin(fmax(p - fl, (Real)0), (Real)1);
        D.k += (int)fl * stride[ax];
        const bool up = w[ax] > (Real)0;
        ks[ax] = mov[ax] ? (up ? stride[ax] : -stride[ax]) : 0;
        dt[ax] = mov[ax] ? fabs(w[ax]) : (Real)INFINITY;
        tn[ax] = mov[ax] ? (up ? (Real)1 - fr : fr) * dt[ax] : (Real)INFINITY;
    }
    D.kx = ks[0];
    D.ky = ks[1];
    D.kz = ks[2];
    D.tx = tn[0];
    D.ty = tn[1];
    D.tz = tn[2];
    D.dtx = dt[0];
    D.dty = dt[1];
    D.dtz = dt[2];
    D.t = (Real)0;
    D.len = (Real)(t1 - t0);
    return ok;
}

// One voxel of a deposit walk.  Every lane of the wavefront runs the
// arithmetic (no branch around it); only busy lanes deposit, and an idle
// lane's walk state is reset by deposit_begin before it is used again.
template <typename Real>
__device__ __forceinline__ void dep_step(DepWalk<Real>& D, double* s_g, double a, uint32_t nloc_b, bool& busy) {
    const int kx = D.kx, ky = D.ky, kz = D.kz;
    const bool cx = (D.tx <= D.ty) && (D.tx <= D.tz);
    const bool cy = !cx && (D.ty <= D.tz);
    const Real tn = fmin(D.tx, fmin(D.ty, D.tz));
    const bool last = tn >= D.len;
    const Real l = (last ? D.len : tn) - D.t;
    if (busy) atomicAdd(reinterpret_cast<double*>(reinterpret_cast<char*>(s_g) + D.k), -a * (double)l);
    D.k += cx ? kx : (cy ? ky : kz);
    D.tx += cx ? D.dtx : (Real)0;
    D.ty += cy ? D.dty : (Real)0;
    D.tz += (!cx && !cy) ? D.dtz : (Real)0;
    D.t = tn;
    // a crossing that rounding put just before the end of the clipped ray
    // must not leave the tile's LDS copy: across a z face the offset leaves
    // the copy's nloc_b bytes, across an x or y face it enters a padding slot (the next
    // crossing of that axis is a voxel further on, past the end)
    busy = busy && !(last || (uint32_t)D.k >= nloc_b);
}

// Each lane keeps the next record it will walk in registers, loaded one
// refill ahead, so that a refill does not wait for memory.
template <typename Real, int TALLY, bool CAMS_LDS>
__global__ void __launch_bounds__(DEPOSIT_BLOCK) k_deposit(KArgs<Real> A, const DepositItem* items) {
    __shared__ double s_g[TILE_LDS];
    __shared__ CamCentre<Real> s_cam[CAMS_LDS ? DEP_LDS_CAMS : 1];
    __shared__ uint32_t s_next;
    const Tape<Real>& P = A.tp;
    const DepositItem it = items[blockIdx.x];
    const int tix = it.tile % P.T.nx, tiy = (it.tile / P.T.nx) % P.T.ny, tiz = it.tile / P.T.nxy;
    const int b0x = tix << P.shx, b0y = tiy << P.shy, b0z = tiz << P.shz;
    DevGrid<Real> L = A.G;
    L.nx = min(1 << P.shx, A.G.nx - b0x);
    L.ny = min(1 << P.shy, A.G.ny - b0y);
    L.nz = min(1 << P.shz, A.G.nz - b0z);
    L.nxy = L.nx * L.ny;
    // padded LDS layout: slot x + px y + pxy z, x <= nx, y <= ny
    const int px = L.nx + 1, pxy = px * (L.ny + 1);
    const int nloc = pxy * L.nz;
    const uint32_t nloc_b = (uint32_t)(sizeof(double) * nloc);
    for (int i = threadIdx.x; i < nloc; i += DEPOSIT_BLOCK) s_g[i] = 0.0;
    for (int i = threadIdx.x; CAMS_LDS && i < A.n_cams; i += DEPOSIT_BLOCK) {
        const DevCam<Real>& cam = A.cams[i];
        CamCentre<Real> cc;
        cc.ix = cam.icx;
        cc.iy = cam.icy;
        cc.iz = cam.icz;
        cc.fx = cam.fcx;
        cc.fy = cam.fcy;
        cc.fz = cam.fcz;
        s_cam[i] = cc;
    }
    // every slot of the tile's bin holds a record (or an empty one)
    const uint32_t hi = it.hi;
    if (threadIdx.x == 0) s_next = it.lo;
    __syncthreads();

    DepWalk<Real> D;
    TapeRec<Real> nxt;
    double a = 0.0;
    bool busy = false, has = false, more = true;
    for (;;) {
        // idle lanes start their prefetched record
        if (!busy && has) {
            busy = deposit_begin<Real, CAMS_LDS>(A, L, px, pxy, b0x, b0y, b0z, s_cam, nxt, s_g, D, a);
            has = false;
        }
        // lanes without a prefetched record take the next slots of the range
        if (more) {
            const unsigned long long want = __ballot(!has);
            if (want) {
                const int leader = __ffsll((long long)want) - 1;
                uint32_t first = 0;
                if (__lane_id() == leader) first = atomicAdd(&s_next, (uint32_t)__popcll(want));
                // the leader's value, read into a scalar register, keeps the
                // loop below uniform for the compiler
                first = __builtin_amdgcn_readlane(first, leader);
                if (first + (uint32_t)__popcll(want) >= hi) more = false;
                if (!has) {
                    const uint32_t s = first + lanes_below(want);
                    if (s < hi) {
                        nxt = P.brec[s];
                        has = true;
                    }
                }
            }
        }
        const bool pending = __ballot(has) != 0ull;
        const uint32_t nbusy = (uint32_t)__popcll(__ballot(busy));
        if (!pending && nbusy == 0) break;
        // walk until a quarter of the lanes are idle while slots are left;
        // after that, until one more lane is idle (a busy lane may hold the
        // last prefetched records), and at the very end until all are
        const uint32_t keep = more ? (uint32_t)WAVE - DEP_REFILL_IDLE : (pending && nbusy > 0 ? nbusy - 1 : 0u);
        while ((uint32_t)__popcll(__ballot(busy)) > keep) {
            // eight voxels per check of the busy count (measured: 4-5% less
            // deposit time than two per check on the 64^3 and 256x256x128
            // workloads; a finished lane steps on with nothing to add)
            dep_step(D, s_g, a, nloc_b, busy);
            dep_step(D, s_g, a, nloc_b, busy);
            dep_step(D, s_g, a, nloc_b, busy);
            dep_step(D, s_g, a, nloc_b, busy);
            dep_step(D, s_g, a, nloc_b, busy);
            dep_step(D, s_g, a, nloc_b, busy);
            dep_step(D, s_g, a, nloc_b, busy);
            dep_step(D, s_g, a, nloc_b, busy);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nloc; i += DEPOSIT_BLOCK) {
        const double v = s_g[i];
        const int x = i % px, y = (i / px) % (L.ny + 1), z = i / pxy;
        if (v != 0.0 && x < L.nx && y < L.ny)
            tally_f64<TALLY>(A.grad, A.grad32, (int64_t)(b0x + x) + (int64_t)A.G.nx * (b0y + y) +
                                                   (int64_t)A.G.nxy * (b0z + z), v);
    }
}

// ---------------------------------------------------------------------------
// Path records: one photon per lane.

template <typename Real>
__device__ __forceinline__ void record_path(const KArgs<Real>& A, uint32_t slot, const Photon<Real>& ph, int fate) {
    mc_path& P = A.paths[slot];
    P.n_events = (int32_t)ph.s;
    P.fate = fate;
    const double te = fate <= MC_FATE_SIDE ? (double)ph.t_exit : 0.0;
    P.exit_pos[0] = absolute(ph.ix, ph.fx, A.G.dx) + te * (double)ph.wx;
    P.exit_pos[1] = absolute(ph.iy, ph.fy, A.G.dy) + te * (double)ph.wy;
    P.exit_pos[2] = absolute(ph.iz, ph.fz, A.G.dz) + te * (double)ph.wz;
    P.exit_dir[0] = (double)ph.wx;
    P.exit_dir[1] = (double)ph.wy;
    P.exit_dir[2] = (double)ph.wz;
    P.exit_w = (double)ph.weight;
}

template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_trace(KArgs<Real> A) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= A.trace_count) return;
    Photon<Real> ph;
    launch_photon(A, A.first_pid + tid, ph);
    uint64_t vfree = 0;
    for (;;) {
        // flights in the render's budgeted pieces, so that a path is the
        // render's to the last rounding
        int left;
        do {
            left = free_flight(A, (const uint32_t*)nullptr, ph, vfree, FLIGHT_BUDGET);
        } while (left == FLIGHT_GOES_ON);
        if (left) {
            record_path(A, tid, ph, left - 1);
            return;
        }
        ph.s += 1;
        int32_t* pix_rec = nullptr;
        if (ph.s <= A.max_rec) {
            const uint64_t e = (uint64_t)tid * A.max_rec + (ph.s - 1);
            mc_event& E = A.ev[e];
            E.x = absolute(ph.ix, ph.fx, A.G.dx);
            E.y = absolute(ph.iy, ph.fy, A.G.dy);
            E.z = absolute(ph.iz, ph.fz, A.G.dz);
            E.w = (double)ph.weight;
            E.voxel = ph.ix + A.G.nx * ph.iy + A.G.nxy * ph.iz;
            E.pad_ = 0;
            if (A.pix) pix_rec = A.pix + e * A.n_cams;
        }
        if (pix_rec) {
            for (int c = 0; c < A.n_cams; ++c) {
                int64_t pix = 0;
                int lp = -1;
                Real vx, vy, vz, r, pre;
                const bool vis = le_geometry(A, A.cams[c], ph.ix, ph.iy, ph.iz, ph.fx, ph.fy, ph.fz, ph.wx, ph.wy,
                                             ph.wz, ph.weight, ph.air, pix, lp, vx, vy, vz, r, pre);
                pix_rec[c] = vis ? lp : -1;
            }
        }
        const int fate = after_collision(A, ph);
        if (fate >= 0) {
            record_path(A, tid, ph, fate);
            return;
        }
    }
}

// ---------------------------------------------------------------------------
// Backward Monte Carlo (Sec. 2.1.4): one packet per lane.

// Transmittance from the collision towards the sun, Eq. (ble): exp(-tau) to
// the top face, 0 when the path leaves through a side face (light enters
// through the top face only, as in the forward method).
template <typename Real>
__device__ __forceinline__ double sun_transmittance(const KArgs<Real>& A, const Photon<Real>& ph) {
    const Real sx = -A.wsx, sy = -A.wsy, sz = -A.wsz;
    const double x = absolute(ph.ix, ph.fx, A.G.dx), y = absolute(ph.iy, ph.fy, A.G.dy);
    const double z = absolute(ph.iz, ph.fz, A.G.dz);
    const double lx = (double)A.G.nx * (double)A.G.dx, ly = (double)A.G.ny * (double)A.G.dy;
    const double tz = ((double)A.G.nz * (double)A.G.dz - z) / (double)sz;
    const double xe = x + tz * (double)sx, ye = y + tz * (double)sy;
    if (!(xe >= 0.0 && xe <= lx && ye >= 0.0 && ye <= ly)) return 0.0;
    ConnWalk<Real> W;
    const Real texit = conn_begin(W, A.G, ph.ix, ph.iy, ph.iz, ph.fx, ph.fy, ph.fz, sx, sy, sz);
    if (texit < (Real)0) return 0.0;
    double tau = 0.0;
    for (;;) {
        bool cx, cy, cz;
        const Real tn = conn_next(W, cx, cy, cz);
        const bool last = tn >= texit;
        tau += (double)A.beta[W.k] * (double)((last ? texit : tn) - W.t);
        if (last) break;
        conn_cross(W, tn, cx, cy, cz);
        if ((uint32_t)W.k >= (uint32_t)A.n_vox) break;
    }
    return exp(-tau);
}

// Packet id p * n_pp + i of global pixel p: leg 0 gives the point of the
// pixel and the first free path; the camera centre and the back-projected
// direction are in double; the packet enters the domain where its ray does.
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_bmc(KArgs<Real> A) {
    __shared__ unsigned long long s_st[ST_N];
    if (threadIdx.x < ST_N) s_st[threadIdx.x] = 0ull;
    __syncthreads();
    uint32_t n_ev = 0;
    uint64_t vfree = 0;
    const Real sx = -A.wsx, sy = -A.wsy, sz = -A.wsz;
    const uint64_t total = (uint64_t)A.n_pix * A.n_pp;
    const double L[3] = {(double)A.G.nx * (double)A.G.dx, (double)A.G.ny * (double)A.G.dy,
                         (double)A.G.nz * (double)A.G.dz};
    const double dv[3] = {(double)A.G.dx, (double)A.G.dy, (double)A.G.dz};
    const int nv[3] = {A.G.nx, A.G.ny, A.G.nz};
    for (uint64_t id = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
         id += (uint64_t)gridDim.x * blockDim.x) {
        const int64_t gp = (int64_t)(id / A.n_pp);
        int lo = 0, hi = A.n_cams - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.hcams[mid].pix_off <= gp) lo = mid;
            else hi = mid - 1;
        }
        const HostCam& cam = A.hcams[lo];
        const int64_t lp = gp - cam.pix_off;
        const int row = (int)(lp / cam.width), col = (int)(lp % cam.width);
        const uint4 r = draw(A.seed, id, 0u);
        const double qx = ((double)col + (double)uniform01<Real>(r.x) - cam.cx) / cam.fx;
        const double qy = ((double)row + (double)uniform01<Real>(r.y) - cam.cy) / cam.fy;
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = cam.R[a] * qx + cam.R[3 + a] * qy + cam.R[6 + a];
        const double il = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        double t0 = 0.0, t1 = INFINITY;
        for (int a = 0; a < 3; ++a) {
            d[a] *= il;
            if (d[a] == 0.0) {
                if (cam.pos[a] < 0.0 || cam.pos[a] > L[a]) t1 = -1.0;
                continue;
            }
            const double ta = (0.0 - cam.pos[a]) / d[a], tb = (L[a] - cam.pos[a]) / d[a];
            t0 = fmax(t0, fmin(ta, tb));
            t1 = fmin(t1, fmax(ta, tb));
        }
        if (!(t1 > t0)) {
            atomicAdd(&s_st[ST_SIDE], 1ull);
            continue;
        }
        Photon<Real> ph;
        int iv[3];
        Real fv[3];
        for (int a = 0; a < 3; ++a) {
            const double f = (cam.pos[a] + t0 * d[a]) / dv[a];
            int i = (int)floor(f);
            if (d[a] < 0.0 && f == floor(f)) i -= 1;
            i = i < 0 ? 0 : (i > nv[a] - 1 ? nv[a] - 1 : i);
            iv[a] = i;
            fv[a] = (Real)(f - (double)i);
        }
        ph.ix = iv[0];
        ph.iy = iv[1];
        ph.iz = iv[2];
        ph.fx = fv[0];
        ph.fy = fv[1];
        ph.fz = fv[2];
        ph.wx = (Real)d[0];
        ph.wy = (Real)d[1];
        ph.wz = (Real)d[2];
        ph.weight = (Real)1;
        ph.taustar = -m_log((Real)1 - uniform01<Real>(r.z));
        ph.t_exit = (Real)0;
        ph.s = 0;
        ph.pid = id;
        ph.air = 0;
        double packet = 0.0;
        for (;;) {
            const int left = free_flight(A, (const uint32_t*)nullptr, ph, vfree, 0xffffffffu);
            if (left) {
                atomicAdd(&s_st[ST_TOP + left - 1], 1ull);
                break;
            }
            ph.s += 1;
            ++n_ev;
            const double t = sun_transmittance(A, ph);
            if (t > 0.0) {
                const Real cosang = ph.wx * sx + ph.wy * sy + ph.wz * sz;
                packet += (double)A.albedo * (double)ph.weight * (double)hg_phase(A.g, cosang) * t;
            }
            const int fate = after_collision(A, ph);
            if (fate >= 0) {
                atomicAdd(&s_st[fate == MC_FATE_CAP ? ST_CAP : ST_RR], 1ull);
                break;
            }
        }
        if (packet != 0.0) {
            unsafeAtomicAdd(A.img + gp, packet / (double)A.n_pp);
            if (A.img_m2) unsafeAtomicAdd(A.img_m2 + gp, packet * packet / (double)A.n_pp);
        }
    }
    if (n_ev) {
        atomicAdd(&s_st[ST_EVENTS], (unsigned long long)n_ev);
        atomicAdd(&s_st[ST_LE], (unsigned long long)n_ev);
    }
    if (vfree) atomicAdd(&s_st[ST_VFREE], (unsigned long long)vfree);
    __syncthreads();
    if (threadIdx.x < ST_N && s_st[threadIdx.x]) atomicAdd(&A.stats[threadIdx.x], s_st[threadIdx.x]);
}

// ---------------------------------------------------------------------------
// Gradient of an air + aerosol mixture with respect to the reference aerosol
// field.  The connection terms come from the MODE_TAPE replay (records with
// weight sig * gw * C, an air collision's marked 0), which for the full
// gradient also sums each collision's a into its photon's row of mix_rows;
// k_mix_path then adds the path scores.  Where the records cannot be binned
// by tile, k_mix_grad does both passes of a photon in one lane.

// Connection ray from (i, f) along unit v over length r (clipped to the
// domain): returns the optical depth, summed voxel by voxel in FP64; with
// DEP, subtracts dep * l(m) from grad in every voxel m.  steps counts the
// voxels visited (one for a walk that cannot start).
template <typename Real, bool DEP>
__device__ double mix_conn(const KArgs<Real>& A, int ix, int iy, int iz, Real fx, Real fy, Real fz, Real vx,
                           Real vy, Real vz, Real r, double dep, uint64_t& steps) {
    ConnWalk<Real> W;
    const Real texit = conn_begin(W, A.G, ix, iy, iz, fx, fy, fz, vx, vy, vz);
    if (texit < (Real)0) {
        ++steps;
        return 0.0;
    }
    const Real rr = fmin(r, texit);
    double tau = 0.0;
    for (;;) {
        bool cx, cy, cz;
        const Real tn = conn_next(W, cx, cy, cz);
        const bool last = tn >= rr;
        const Real l = (last ? rr : tn) - W.t;
        ++steps;
        tau += (double)A.beta[W.k] * (double)l;
        if (DEP) unsafeAtomicAdd(A.grad + W.k, -dep * (double)l);
        conn_cross(W, tn, cx, cy, cz);
        if (last || (uint32_t)W.k >= (uint32_t)A.n_vox) break;
    }
    return tau;
}

// The connection term of one local estimate (sa = sig * a): a ray record for
// the tile bins, whose deposit kernel adds -sa l(m) along the ray and, for
// an aerosol collision, sa / beta_aer at its start (k_bin, k_deposit); when
// the wavefront's slice is full, or the grid has no tiles, the same terms
// go straight to grad with device atomics.
template <typename Real>
__device__ void mix_record(const KArgs<Real>& A, uint32_t* s_wc, const Photon<Real>& ph, int64_t pix, double sa,
                           int64_t ke, Real vx, Real vy, Real vz, Real r) {
    if (A.tape) {
        const uint32_t slot = atomicAdd(&s_wc[threadIdx.x / WAVE], 1u);
        if (slot < A.tp.rw) {
            TapeRec<Real> R;
            R.vox = (uint32_t)ph.ix | ((uint32_t)ph.iy << 11) | ((uint32_t)ph.iz << 22);
            R.id = (uint32_t)pix;
            R.fx = ph.fx;
            R.fy = ph.fy;
            R.fz = ph.fz;
            R.a = (Real)sa;
            R.ab = ph.air ? (Real)0 : (Real)1;
            const size_t w = (size_t)blockIdx.x * (BLOCK / WAVE) + threadIdx.x / WAVE;
            A.tp.rec[w * A.tp.rw + slot] = R;
            return;
        }
    }
    uint64_t dummy = 0;
    if (!ph.air) unsafeAtomicAdd(A.grad + ke, sa / __dmul_rn(A.mix_sig, A.mix_aer[ke]));
    mix_conn<Real, true>(A, ph.ix, ph.iy, ph.iz, ph.fx, ph.fy, ph.fz, vx, vy, vz, r, sa, dummy);
}

// One leg of a photon: its free flight and, if it collides, the collision;
// returns false when the photon has left or ended.  PASS 0: the surrogate
// (in-scatter field frozen): every estimate's connection term (mix_record).
// PASS 1: the same, and the sum of a = dL/di norm C over the photon's
// estimates (asum; any: some a is not zero), keeping the sums of its first
// mix_evcap collisions in ev_row.  PASS 2: the path scores of the full
// gradient with ffd = sig * A_s, A_s the sum of a over collisions s and
// later (the photon's whole sum at the start): the free-flight terms
// -ffd l, at an aerosol collision (ffd - sig a_s) / beta_aer (the
// collision's own estimates are in their records), then A_s minus this
// collision's a (read back from ev_row, or its estimates walked again past
// the first mix_evcap collisions).
template <typename Real, int PASS>
__device__ __forceinline__ bool mix_leg(const KArgs<Real>& A, Photon<Real>& ph, double& ffd, double* ev_row,
                                        double& asum, bool& any, unsigned long long* s_st, uint32_t* s_wc,
                                        uint64_t& n_ev, uint64_t& n_le, uint64_t& vfree, uint64_t& vconn) {
    constexpr bool COUNT = PASS != 2;
    uint64_t dummy = 0;
    const int left = free_flight<Real, PASS == 2>(A, (const uint32_t*)nullptr, ph, COUNT ? vfree : dummy,
                                                  0xffffffffu, ffd, A.grad);
    if (left) {
        if (COUNT) atomicAdd(&s_st[ST_TOP + left - 1], 1ull);
        return false;
    }
    ph.s += 1;
    if (COUNT) ++n_ev;
    ph.air = mix_particle(A, ph);
    const int64_t ke = (int64_t)ph.ix + (int64_t)A.G.nx * ph.iy + (int64_t)A.G.nxy * ph.iz;
    double ev_a = 0.0;
    const bool kept = ev_row && ph.s <= A.mix_evcap;
    if (PASS == 2 && kept) ev_a = ev_row[ph.s - 1];
    for (int c = 0; c < A.n_cams && !(PASS == 2 && kept); ++c) {
        int64_t pix = 0;
        int lp = 0;
        Real vx = 0, vy = 0, vz = 0, r = 0, pre = 0;
        if (!le_geometry(A, A.cams[c], ph.ix, ph.iy, ph.iz, ph.fx, ph.fy, ph.fz, ph.wx, ph.wy, ph.wz, ph.weight,
                         ph.air, pix, lp, vx, vy, vz, r, pre))
            continue;
        if (COUNT) ++n_le;
        const double tau = mix_conn<Real, false>(A, ph.ix, ph.iy, ph.iz, ph.fx, ph.fy, ph.fz, vx, vy, vz, r, 0.0,
                                                 COUNT ? vconn : dummy);
        const double C = (double)pre * (double)m_exp((Real)(-tau));
        const double a = A.gw[pix] * C;
        if (PASS == 1) {
            asum += a;
            any = any || a != 0.0;
        }
        if (PASS != 0) ev_a += a;
        if (PASS != 2 && a != 0.0) mix_record(A, s_wc, ph, pix, A.mix_sig * a, ke, vx, vy, vz, r);
    }
    if (PASS == 1 && kept) ev_row[ph.s - 1] = ev_a;
    if (PASS == 2) {
        const double later = ffd - A.mix_sig * ev_a;
        if (!ph.air && later != 0.0) unsafeAtomicAdd(A.grad + ke, later / __dmul_rn(A.mix_sig, A.mix_aer[ke]));
        ffd = later;
    }
    const int fate = after_collision(A, ph);
    if (fate >= 0) {
        if (COUNT) atomicAdd(&s_st[fate == MC_FATE_CAP ? ST_CAP : ST_RR], 1ull);
        return false;
    }
    return true;
}

// One photon, all of its legs in one lane (see mix_leg).
template <typename Real, int PASS>
__device__ void mix_photon(const KArgs<Real>& A, uint64_t pid, double ffd, double* ev_row, double& asum, bool& any,
                           unsigned long long* s_st, uint32_t* s_wc, uint64_t& n_ev, uint64_t& n_le, uint64_t& vfree,
                           uint64_t& vconn) {
    Photon<Real> ph;
    launch_photon(A, pid, ph);
    while (mix_leg<Real, PASS>(A, ph, ffd, ev_row, asum, any, s_st, s_wc, n_ev, n_le, vfree, vconn)) {
    }
}

template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_mix_grad(KArgs<Real> A) {
    __shared__ unsigned long long s_st[ST_N];
    __shared__ uint32_t s_wc[BLOCK / WAVE];  // records written per wavefront
    if (threadIdx.x < ST_N) s_st[threadIdx.x] = 0ull;
    if (threadIdx.x < BLOCK / WAVE) s_wc[threadIdx.x] = 0u;
    __syncthreads();
    uint64_t n_ev = 0, n_le = 0, vfree = 0, vconn = 0;
    for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < A.n_photons;
         k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t pid = A.pid0 + k;
        double asum = 0.0;
        bool any = false;
        double* row = A.mix_evs ? A.mix_evs + ((size_t)blockIdx.x * blockDim.x + threadIdx.x) * A.mix_evcap : nullptr;
        if (!A.mix_full) {
            mix_photon<Real, 0>(A, pid, 0.0, nullptr, asum, any, s_st, s_wc, n_ev, n_le, vfree, vconn);
        } else {
            mix_photon<Real, 1>(A, pid, 0.0, row, asum, any, s_st, s_wc, n_ev, n_le, vfree, vconn);
            if (any)
                mix_photon<Real, 2>(A, pid, A.mix_sig * asum, row, asum, any, s_st, s_wc, n_ev, n_le, vfree, vconn);
        }
    }
    if (n_ev) atomicAdd(&s_st[ST_EVENTS], (unsigned long long)n_ev);
    if (n_le) atomicAdd(&s_st[ST_LE], (unsigned long long)n_le);
    if (vfree) atomicAdd(&s_st[ST_VFREE], (unsigned long long)vfree);
    if (vconn) atomicAdd(&s_st[ST_VCONN], (unsigned long long)vconn);
    __syncthreads();
    if (threadIdx.x < ST_N && s_st[threadIdx.x]) atomicAdd(&A.stats[threadIdx.x], s_st[threadIdx.x]);
    if (A.tape && threadIdx.x < BLOCK / WAVE) A.tp.wave_count[blockIdx.x * (BLOCK / WAVE) + threadIdx.x] = s_wc[threadIdx.x];
}

// Path scores of the full gradient after the tape replay of the same photons
// (which deposited the connection terms): photon k of the launch has in row
// k of mix_rows the sums of a over the estimates of its collisions 1 ..
// mix_evcap and, in the last entry, over all later ones; A_s starts at the
// row's sum.  Past the first mix_evcap collisions the estimates are walked
// again.  One leg per pass of the loop, as in the forward: a lane whose
// photon ends takes its next photon with a non-zero row at once, instead of
// waiting for the wavefront's longest photon.  No counters (the replay
// counted the photons).
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_mix_path(KArgs<Real> A) {
    uint64_t dummy = 0;
    const uint32_t w = A.mix_evcap + 1u;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;  // the lane's next photon
    Photon<Real> ph;
    double ffd = 0.0, asum = 0.0;
    double* row = nullptr;
    bool alive = false, any = false;
    for (;;) {
        while (!alive && k < A.n_photons) {
            row = A.mix_rows + k * w;
            asum = 0.0;
            any = false;
            for (uint32_t j = 0; j < w; ++j) {
                asum += row[j];
                any = any || row[j] != 0.0;
            }
            if (any) {
                launch_photon(A, A.pid0 + k, ph);
                ffd = A.mix_sig * asum;
                alive = true;
            }
            k += stride;
        }
        if (__ballot(alive) == 0ull) break;
        if (alive)
            alive = mix_leg<Real, 2>(A, ph, ffd, row, asum, any, nullptr, nullptr, dummy, dummy, dummy, dummy);
    }
}

// The channel's extinction beta = air + sig * aer (reference aerosol field
// times the channel's cross-section ratio, Eq. channelBeta) in the kernels'
// precision, rounded step by step (no fused multiply-add), followed by the
// zeros of the library's copy.
template <typename Real>
__global__ void k_mix_total(Real* beta, const double* air, const double* aer, double sig, int64_t n, int64_t pad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) beta[i] = (Real)__dadd_rn(air[i], __dmul_rn(sig, aer[i]));
    else if (i < n + pad) beta[i] = (Real)0;
}

// ---------------------------------------------------------------------------
// small kernels

template <typename Real>
__global__ void k_write_cams(CamChunk chunk, DevCam<Real>* dev, NormCam* norm) {
    const int i = threadIdx.x;
    if (i >= chunk.n) return;
    const HostCam& h = chunk.c[i];
    DevCam<Real> d;
    // camera centre in voxel units, split into integer and fraction
    const double pcx = h.pos[0] / chunk.dx, pcy = h.pos[1] / chunk.dy, pcz = h.pos[2] / chunk.dz;
    const double ix = floor(pcx), iy = floor(pcy), iz = floor(pcz);
    d.icx = (int32_t)ix;
    d.icy = (int32_t)iy;
    d.icz = (int32_t)iz;
    d.fcx = (Real)(pcx - ix);
    d.fcy = (Real)(pcy - iy);
    d.fcz = (Real)(pcz - iz);
    d.pad_ = 0;
    d.pfcx = pcx - ix;
    d.pfcy = pcy - iy;
    d.pfcz = pcz - iz;
    for (int j = 0; j < 9; ++j) d.R[j] = h.R[j];
    d.fx = h.fx;
    d.fy = h.fy;
    d.cx = h.cx;
    d.cy = h.cy;
    d.fw = (double)h.width;
    d.fh = (double)h.height;
    d.width = h.width;
    d.pix_off = (int32_t)h.pix_off;
    dev[chunk.first + i] = d;
    NormCam n;
    n.fx = h.fx;
    n.fy = h.fy;
    n.cx = h.cx;
    n.cy = h.cy;
    n.width = h.width;
    n.height = h.height;
    n.pix_off = h.pix_off;
    norm[chunk.first + i] = n;
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}
__global__ void k_fill_f64(double* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}
__global__ void k_fill_f32(float* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}
// Eq. (Jc): j = L * base / beta, 0 where beta = 0 (base = mu0 A_top / N);
// L is laid out [voxel][pitch], j [camera][voxel].
template <typename Real>
__global__ void k_voxel_finish(double* j, const double* L, int pitch, const Real* beta, int n_cams, int64_t n_vox,
                               double base) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n_vox; k += (int64_t)gridDim.x * blockDim.x) {
        const double b = (double)beta[k];
        const double* Lk = L + k * pitch;
        for (int c = 0; c < n_cams; ++c) j[(int64_t)c * n_vox + k] = b > 0.0 ? Lk[c] * base / b : 0.0;
    }
}

__global__ void k_fill_u32(uint32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Solid angle of a pixel: the rectangle [x1,x2] x [y1,y2] on the unit-focal
// plane subtends F(x2,y2) - F(x1,y2) - F(x2,y1) + F(x1,y1) with
// F(x, y) = atan(x y / sqrt(1 + x^2 + y^2)).
__device__ __forceinline__ double rect_solid_angle(double x1, double x2, double y1, double y2) {
    auto F = [](double x, double y) { return atan(x * y / sqrt(1.0 + x * x + y * y)); };
    return F(x2, y2) - F(x1, y2) - F(x2, y1) + F(x1, y1);
}

// mu0 A_top / (N Omega_p) of pixel p.
__device__ __forceinline__ double pixel_norm(const NormCam* cams, int n_cams, int64_t p, double base) {
    int c = 0;
    while (c + 1 < n_cams && cams[c + 1].pix_off <= p) ++c;
    const NormCam& K = cams[c];
    const int64_t local = p - K.pix_off;
    const int row = (int)(local / K.width), col = (int)(local % K.width);
    const double om = rect_solid_angle((col - K.cx) / K.fx, (col + 1 - K.cx) / K.fx, (row - K.cy) / K.fy,
                                       (row + 1 - K.cy) / K.fy);
    return base / om;
}

__global__ void k_normalize(double* img, const NormCam* cams, int n_cams, int64_t n_pix, double base, int power) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n_pix) {
        const double n = pixel_norm(cams, n_cams, p, base);
        img[p] *= power == 2 ? n * n : n;
    }
}

__global__ void k_grad_weights(double* gw, const double* dl, const NormCam* cams, int n_cams, int64_t n_pix,
                               double base) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n_pix) gw[p] = dl[p] * pixel_norm(cams, n_cams, p, base);
}

// One 32-bit word of the occupancy bitmask per thread: bit j of word w is
// set when a voxel of run 32 w + j has beta > 0 (or a non-finite beta,
// which must reach the walk unchanged).
template <typename Real>
__global__ void k_build_mask(KArgs<Real> A, uint32_t* mask) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= A.mask_words) return;
    uint32_t word = 0;
    for (int j = 0; j < 32; ++j) {
        const int64_t k0 = ((int64_t)w * 32 + j) << A.msh;
        const int64_t k1 = min(k0 + ((int64_t)1 << A.msh), A.n_vox);
        bool any = false;
        for (int64_t k = k0; k < k1 && !any; ++k) any = !(A.beta[k] == (Real)0) || !(A.beta_le[k] == (Real)0);
        if (any) word |= 1u << j;
    }
    mask[w] = word;
}

// Occupancy mask of a mixture whose air depends on the height only: runs
// holding aerosol (aer > 0); the air of the other voxels is the column's.
template <typename Real>
__global__ void k_build_mask_aer(KArgs<Real> A, uint32_t* mask) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= A.mask_words) return;
    uint32_t word = 0;
    for (int j = 0; j < 32; ++j) {
        const int64_t k0 = ((int64_t)w * 32 + j) << A.msh;
        const int64_t k1 = min(k0 + ((int64_t)1 << A.msh), A.n_vox);
        bool any = false;
        for (int64_t k = k0; k < k1 && !any; ++k) any = !(A.mix_aer[k] == 0.0);
        if (any) word |= 1u << j;
    }
    mask[w] = word;
}

// Air column of a mixture: col[iz] = the channel's extinction of an
// aerosol-free voxel of layer iz (the value the library's copy of beta holds
// there), and flag != 0 when some voxel's air differs from its layer's
// first voxel (the air is then not a function of the height alone).
template <typename Real>
__global__ void k_air_column(const double* air, int64_t n_vox, int64_t nxy, int nz, Real* col, uint32_t* flag) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nz) col[k] = (Real)air[k * nxy];
    const bool diff = k < n_vox && !(air[k] == air[(k / nxy) * nxy]);
    if (__ballot(diff) != 0ull && __lane_id() == 0) atomicOr(flag, 1u);
}

__global__ void k_kahan_reduce(double* out, const float* pairs, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)pairs[2 * i] + (double)pairs[2 * i + 1];
}

// ---------------------------------------------------------------------------
// launchers

static inline int blocks_for(int64_t n) { return (int)((n + BLOCK - 1) / BLOCK); }

template <typename Real>
hipError_t launch_write_cams(const CamChunk& chunk, DevCam<Real>* dev, NormCam* norm, hipStream_t s) {
    hipLaunchKernelGGL(k_write_cams<Real>, dim3(1), dim3(64), 0, s, chunk, dev, norm);
    return hipGetLastError();
}

// Dynamic LDS bytes of k_render for these arguments.
template <typename Real>
size_t render_dyn_lds(const KArgs<Real>& a, int mode) {
    size_t words = (size_t)((a.mask_words + 1) & ~1);
    size_t bytes = words * sizeof(uint32_t);
    if (mode == MODE_GRAD && a.grad_lds) bytes += (size_t)a.n_vox * sizeof(double);
    return bytes;
}

template <typename Real, int MODE, int TALLY, bool AIRZ = false, bool W32 = false, bool CAP = false>
static hipError_t launch_r(const KArgs<Real>& a, int grid, hipStream_t s) {
    const size_t dyn = render_dyn_lds(a, MODE);
    KArgs<Real> b = a;
    const uint64_t waves = (uint64_t)std::max(grid, 1) * (RenderThreads<MODE>::value / WAVE);
    b.fetch_block = (uint32_t)std::min<uint64_t>(FETCH_BLOCK_MAX, std::max<uint64_t>(WAVE, a.n_photons / (32 * waves)));
    hipLaunchKernelGGL((k_render<Real, MODE, TALLY, AIRZ, W32, CAP>), dim3(grid), dim3(RenderThreads<MODE>::value),
                       dyn, s, b);
    return hipGetLastError();
}

hipError_t launch_capture(const KArgs<float>& a, int grid, hipStream_t s) {
    return launch_r<float, MODE_RENDER, TALLY_F64, false, false, true>(a, grid, s);
}

template <typename Real>
hipError_t launch_mix_path(const KArgs<Real>& a, int grid, hipStream_t s) {
    if (grid > 0) hipLaunchKernelGGL(k_mix_path<Real>, dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

// The connection walks read beta with plain loads (the AIRZ kernels) when
// empty runs read an air column, or when the voxels exceed the range of the
// walks' buffer (then air_step = 0: the air column is the zero word).
template <typename Real>
static bool plain_walk(const KArgs<Real>& a) {
    return a.air_step != 0 || !a.walk_buf;
}

template <typename Real>
hipError_t launch_transport(const KArgs<Real>& a, int mode, int tally, int grid, hipStream_t s) {
    const bool plain = plain_walk(a);
    if constexpr (sizeof(Real) == 8) {
        if (mode == MODE_RENDER && a.walk32 && plain)
            return tally == TALLY_F64 ? launch_r<Real, MODE_RENDER, TALLY_F64, true, true>(a, grid, s)
                                      : launch_r<Real, MODE_RENDER, TALLY_K32, true, true>(a, grid, s);
        if (mode == MODE_RENDER && a.walk32)
            return tally == TALLY_F64 ? launch_r<Real, MODE_RENDER, TALLY_F64, false, true>(a, grid, s)
                                      : launch_r<Real, MODE_RENDER, TALLY_K32, false, true>(a, grid, s);
    }
    if (mode == MODE_RENDER && plain) {
        return tally == TALLY_F64 ? launch_r<Real, MODE_RENDER, TALLY_F64, true>(a, grid, s)
                                  : launch_r<Real, MODE_RENDER, TALLY_K32, true>(a, grid, s);
    }
    if (mode == MODE_RENDER) {
        return tally == TALLY_F64 ? launch_r<Real, MODE_RENDER, TALLY_F64>(a, grid, s)
                                  : launch_r<Real, MODE_RENDER, TALLY_K32>(a, grid, s);
    }
    if (mode == MODE_GRAD) {
        return tally == TALLY_F64 ? launch_r<Real, MODE_GRAD, TALLY_F64>(a, grid, s)
                                  : launch_r<Real, MODE_GRAD, TALLY_K32>(a, grid, s);
    }
    if (mode == MODE_TAPE)
        return plain ? launch_r<Real, MODE_TAPE, TALLY_F64, true>(a, grid, s)
                     : launch_r<Real, MODE_TAPE, TALLY_F64>(a, grid, s);
    if (mode == MODE_RTAPE && plain) {
        return tally == TALLY_F64 ? launch_r<Real, MODE_RTAPE, TALLY_F64, true>(a, grid, s)
                                  : launch_r<Real, MODE_RTAPE, TALLY_K32, true>(a, grid, s);
    }
    if (mode == MODE_RTAPE) {
        return tally == TALLY_F64 ? launch_r<Real, MODE_RTAPE, TALLY_F64>(a, grid, s)
                                  : launch_r<Real, MODE_RTAPE, TALLY_K32>(a, grid, s);
    }
    if (mode == MODE_VOXEL) return launch_r<Real, MODE_VOXEL, TALLY_F64>(a, grid, s);
    if (mode == MODE_BMC) {
        hipLaunchKernelGGL(k_bmc<Real>, dim3(grid), dim3(BLOCK), 0, s, a);
        return hipGetLastError();
    }
    if (mode == MODE_MIXGRAD) {
        hipLaunchKernelGGL(k_mix_grad<Real>, dim3(grid), dim3(BLOCK), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_trace<Real>, dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <typename Real, int MODE, int TALLY, bool AIRZ = false, bool W32 = false>
static hipError_t occ_r(const KArgs<Real>& a, int* b) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(b, (const void*)k_render<Real, MODE, TALLY, AIRZ, W32>,
                                                        RenderThreads<MODE>::value, render_dyn_lds(a, MODE));
}

template <typename Real>
hipError_t transport_occupancy(const KArgs<Real>& a, int mode, int tally, int* b) {
    const bool plain = plain_walk(a);
    if constexpr (sizeof(Real) == 8) {
        if (mode == MODE_RENDER && a.walk32 && plain)
            return tally == TALLY_F64 ? occ_r<Real, MODE_RENDER, TALLY_F64, true, true>(a, b)
                                      : occ_r<Real, MODE_RENDER, TALLY_K32, true, true>(a, b);
        if (mode == MODE_RENDER && a.walk32)
            return tally == TALLY_F64 ? occ_r<Real, MODE_RENDER, TALLY_F64, false, true>(a, b)
                                      : occ_r<Real, MODE_RENDER, TALLY_K32, false, true>(a, b);
    }
    if (mode == MODE_RENDER && plain)
        return tally == TALLY_F64 ? occ_r<Real, MODE_RENDER, TALLY_F64, true>(a, b)
                                  : occ_r<Real, MODE_RENDER, TALLY_K32, true>(a, b);
    if (mode == MODE_RENDER) return tally == TALLY_F64 ? occ_r<Real, MODE_RENDER, TALLY_F64>(a, b)
                                                       : occ_r<Real, MODE_RENDER, TALLY_K32>(a, b);
    if (mode == MODE_GRAD) return tally == TALLY_F64 ? occ_r<Real, MODE_GRAD, TALLY_F64>(a, b)
                                                     : occ_r<Real, MODE_GRAD, TALLY_K32>(a, b);
    if (mode == MODE_TAPE)
        return plain ? occ_r<Real, MODE_TAPE, TALLY_F64, true>(a, b) : occ_r<Real, MODE_TAPE, TALLY_F64>(a, b);
    if (mode == MODE_RTAPE && plain)
        return tally == TALLY_F64 ? occ_r<Real, MODE_RTAPE, TALLY_F64, true>(a, b)
                                  : occ_r<Real, MODE_RTAPE, TALLY_K32, true>(a, b);
    if (mode == MODE_RTAPE) return tally == TALLY_F64 ? occ_r<Real, MODE_RTAPE, TALLY_F64>(a, b)
                                                      : occ_r<Real, MODE_RTAPE, TALLY_K32>(a, b);
    if (mode == MODE_VOXEL) return occ_r<Real, MODE_VOXEL, TALLY_F64>(a, b);
    if (mode == MODE_BMC) return hipOccupancyMaxActiveBlocksPerMultiprocessor(b, (const void*)k_bmc<Real>, BLOCK, 0);
    if (mode == MODE_MIXGRAD)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(b, (const void*)k_mix_grad<Real>, BLOCK, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(b, (const void*)k_trace<Real>, BLOCK, 0);
}

template <typename Real>
hipError_t launch_voxel_finish(double* j, const double* L, int pitch, const Real* beta, int n_cams, int64_t n_vox,
                               double base, hipStream_t s) {
    const int grid = (int)std::min<int64_t>((n_vox + BLOCK - 1) / BLOCK, 65536);
    if (grid > 0)
        hipLaunchKernelGGL(k_voxel_finish<Real>, dim3(grid), dim3(BLOCK), 0, s, j, L, pitch, beta, n_cams, n_vox, base);
    return hipGetLastError();
}

template hipError_t launch_voxel_finish<float>(double*, const double*, int, const float*, int, int64_t, double,
                                               hipStream_t);
template hipError_t launch_voxel_finish<double>(double*, const double*, int, const double*, int, int64_t, double,
                                                hipStream_t);

template <typename Real>
hipError_t launch_build_mask(const KArgs<Real>& a, uint32_t* mask, hipStream_t s) {
    hipLaunchKernelGGL(k_build_mask<Real>, dim3(blocks_for(a.mask_words)), dim3(BLOCK), 0, s, a, mask);
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_build_mask_aer(const KArgs<Real>& a, uint32_t* mask, hipStream_t s) {
    hipLaunchKernelGGL(k_build_mask_aer<Real>, dim3(blocks_for(a.mask_words)), dim3(BLOCK), 0, s, a, mask);
    return hipGetLastError();
}
template hipError_t launch_build_mask_aer<float>(const KArgs<float>&, uint32_t*, hipStream_t);
template hipError_t launch_build_mask_aer<double>(const KArgs<double>&, uint32_t*, hipStream_t);

template <typename Real>
hipError_t launch_air_column(const double* air, int64_t n_vox, int64_t nxy, int nz, Real* col, uint32_t* flag,
                             hipStream_t s) {
    const int64_t n = n_vox > nz ? n_vox : nz;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_air_column<Real>, dim3(blocks_for(n)), dim3(BLOCK), 0, s, air, n_vox, nxy, nz, col, flag);
    return hipGetLastError();
}
template hipError_t launch_air_column<float>(const double*, int64_t, int64_t, int, float*, uint32_t*, hipStream_t);
template hipError_t launch_air_column<double>(const double*, int64_t, int64_t, int, double*, uint32_t*,
                                              hipStream_t);

template <typename Real>
hipError_t launch_bin(const KArgs<Real>& a, bool scatter, hipStream_t s) {
    const int grid = a.tp.n_slices;  // split blocks per wavefront slice
    if (grid <= 0) return hipSuccess;
    const size_t tiles = scatter ? (size_t)(a.tp.t_hi - a.tp.t_lo) : (size_t)a.tp.n_tiles;
    const size_t dyn = sizeof(uint32_t) * ((size_t)std::min(a.n_cams, BIN_LDS_CAMS) + (scatter ? 3 : 1) * tiles);
    hipLaunchKernelGGL(k_bin<Real>, dim3(grid), dim3(BLOCK), dyn, s, a, scatter ? 1 : 0);
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_bin_scan(const KArgs<Real>& a, hipStream_t s) {
    if (a.tp.t_hi <= a.tp.t_lo) return hipSuccess;
    hipLaunchKernelGGL(k_bin_scan<Real>, dim3(a.tp.t_hi - a.tp.t_lo), dim3(SCAN_BLOCK), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_bin<float>(const KArgs<float>&, bool, hipStream_t);
template hipError_t launch_bin<double>(const KArgs<double>&, bool, hipStream_t);
template hipError_t launch_bin_scan<float>(const KArgs<float>&, hipStream_t);
template hipError_t launch_bin_scan<double>(const KArgs<double>&, hipStream_t);

template <typename Real>
hipError_t launch_deposit(const KArgs<Real>& a, int tally, const DepositItem* items, int n_items, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    const bool lds = a.n_cams <= DEP_LDS_CAMS;
    if (tally == TALLY_F64 && lds)
        hipLaunchKernelGGL((k_deposit<Real, TALLY_F64, true>), dim3(n_items), dim3(DEPOSIT_BLOCK), 0, s, a, items);
    else if (tally == TALLY_F64)
        hipLaunchKernelGGL((k_deposit<Real, TALLY_F64, false>), dim3(n_items), dim3(DEPOSIT_BLOCK), 0, s, a, items);
    else if (lds)
        hipLaunchKernelGGL((k_deposit<Real, TALLY_K32, true>), dim3(n_items), dim3(DEPOSIT_BLOCK), 0, s, a, items);
    else
        hipLaunchKernelGGL((k_deposit<Real, TALLY_K32, false>), dim3(n_items), dim3(DEPOSIT_BLOCK), 0, s, a, items);
    return hipGetLastError();
}

template hipError_t launch_deposit<float>(const KArgs<float>&, int, const DepositItem*, int, hipStream_t);
template hipError_t launch_deposit<double>(const KArgs<double>&, int, const DepositItem*, int, hipStream_t);
template hipError_t launch_build_mask<float>(const KArgs<float>&, uint32_t*, hipStream_t);
template hipError_t launch_build_mask<double>(const KArgs<double>&, uint32_t*, hipStream_t);
template hipError_t launch_write_cams<float>(const CamChunk&, DevCam<float>*, NormCam*, hipStream_t);
template hipError_t launch_write_cams<double>(const CamChunk&, DevCam<double>*, NormCam*, hipStream_t);
template <typename Real>
hipError_t launch_mix_total(Real* beta, const double* air, const double* aer, double sig, int64_t n, int64_t pad,
                            hipStream_t s) {
    const int64_t m = n + pad;
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mix_total<Real>, dim3(blocks_for(m)), dim3(BLOCK), 0, s, beta, air, aer, sig, n, pad);
    return hipGetLastError();
}
template hipError_t launch_mix_total<float>(float*, const double*, const double*, double, int64_t, int64_t,
                                            hipStream_t);
template hipError_t launch_mix_total<double>(double*, const double*, const double*, double, int64_t, int64_t,
                                             hipStream_t);

template hipError_t launch_mix_path<float>(const KArgs<float>&, int, hipStream_t);
template hipError_t launch_mix_path<double>(const KArgs<double>&, int, hipStream_t);
template hipError_t launch_transport<float>(const KArgs<float>&, int, int, int, hipStream_t);
template hipError_t launch_transport<double>(const KArgs<double>&, int, int, int, hipStream_t);
template hipError_t transport_occupancy<float>(const KArgs<float>&, int, int, int*);
template hipError_t transport_occupancy<double>(const KArgs<double>&, int, int, int*);

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n)), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks_for(n)), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks_for(n)), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n)), dim3(BLOCK), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_normalize(double* img, const NormCam* cams, int n_cams, int64_t n_pix, double base, int power,
                            hipStream_t s) {
    if (n_pix <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_normalize, dim3(blocks_for(n_pix)), dim3(BLOCK), 0, s, img, cams, n_cams, n_pix, base,
                       power);
    return hipGetLastError();
}
hipError_t launch_grad_weights(double* gw, const double* dl, const NormCam* cams, int n_cams, int64_t n_pix,
                               double base, hipStream_t s) {
    if (n_pix <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_weights, dim3(blocks_for(n_pix)), dim3(BLOCK), 0, s, gw, dl, cams, n_cams, n_pix,
                       base);
    return hipGetLastError();
}
hipError_t launch_kahan_reduce(double* out, const float* pairs, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_kahan_reduce, dim3(blocks_for(n)), dim3(BLOCK), 0, s, out, pairs, n);
    return hipGetLastError();
}

}  // namespace mcrt
