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
// Large grids write the ray to a tape instead, once per gradient tile it
// crosses, and k_deposit accumulates every tile's rays in LDS: a device-scope
// atomic add per voxel crossing would run at the memory-side atomic rate,
// far below the walk.
//
// k_trace: one photon per lane, the same transport, recording events.
#include "mcrt_internal.hpp"

namespace mcrt {

constexpr int WAVE = 64;
constexpr int WAVES = BLOCK / WAVE;
constexpr uint32_t QCAP = 128;     // local-estimate jobs per wavefront queue
constexpr uint32_t REFILL_IDLE = 16;

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
};

// Absolute coordinate (km) of a voxel-local position.
template <typename Real>
__device__ __forceinline__ double absolute(int i, Real f, Real d) {
    return ((double)i + (double)f) * (double)d;
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long mask) {
    return (uint32_t)__popcll(mask & __lanemask_lt());
}

// The active lanes take consecutive photon ids with one atomic.
__device__ __forceinline__ uint64_t wave_fetch(unsigned long long* work) {
    const unsigned long long mask = __ballot(1);
    const int leader = __ffsll((long long)mask) - 1;
    unsigned long long base = 0;
    if (__lane_id() == leader) base = atomicAdd(work, (unsigned long long)__popcll(mask));
    const unsigned lo = __shfl((unsigned)base, leader);
    const unsigned hi = __shfl((unsigned)(base >> 32), leader);
    return (((uint64_t)hi << 32) | lo) + lanes_below(mask);
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

// Occupancy of the voxel (ix, iy, iz) / linear k in the bitmask of cells
// that hold a non-zero extinction: an empty voxel contributes nothing to any
// optical depth, so its extinction need not be fetched.
template <typename Real>
__device__ __forceinline__ bool occupied(const KArgs<Real>& A, const uint32_t* mask, int ix, int iy, int iz, int k) {
    const uint32_t cell = A.mask_fine ? (uint32_t)k
                                      : (uint32_t)((ix >> A.mshx) + A.mncx * ((iy >> A.mshy) + A.mncy * (iz >> A.mshz)));
    return (mask[cell >> 5] >> (cell & 31u)) & 1u;
}

// Extinction of the walk's current voxel, or 0 without a fetch when its cell
// is empty (no mask: always fetched).
template <typename Real>
__device__ __forceinline__ Real beta_at(const KArgs<Real>& A, const uint32_t* mask, const WalkRegs<Real>& W) {
    if (mask && !occupied(A, mask, W.ix, W.iy, W.iz, W.k)) return (Real)0;
    return A.beta[W.k];
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
}

// Steps (ii)-(iii): returns 0 on a collision (position and voxel updated),
// else 1 + face code (0 top, 1 bottom, 2 side), with the position unchanged
// and t_exit set.  The extinction of the next voxel is loaded one crossing
// ahead of its use.
template <typename Real>
__device__ __forceinline__ int free_flight(const KArgs<Real>& A, const uint32_t* mask, Photon<Real>& ph,
                                           uint64_t& vfree) {
    WalkRegs<Real> W;
    const Real f0x = ph.fx, f0y = ph.fy, f0z = ph.fz;
    const Real wx = ph.wx, wy = ph.wy, wz = ph.wz;
    const Real taustar = ph.taustar;
    if (!walk_begin(W, A.G, ph.ix, ph.iy, ph.iz, f0x, f0y, f0z, wx, wy, wz)) {
        ph.t_exit = (Real)0;
        return 3;
    }
    Real tau = (Real)0, tc = (Real)0;
    Real b = beta_at(A, mask, W);
    uint32_t steps = 0;
    int left = 0;
    for (;;) {
        ++steps;
        bool cx, cy, cz;
        const Real tn = walk_next(W, cx, cy, cz);
        const Real seg = tn - W.t;
        if (b > (Real)0 && tau + b * seg >= taustar) {
            tc = W.t + (taustar - tau) / b;
            break;
        }
        tau += b * seg;
        const bool out = walk_cross(W, A.G, tn, cx, cy, cz);
        if (out) {
            left = cz ? (W.sz > 0 ? 1 : 2) : 3;
            break;
        }
        b = beta_at(A, mask, W);
    }
    vfree += steps;
    if (left == 0) {
        ph.fx = walk_frac(f0x, W.sfx, W.rx, wx, A.G.idx, tc);
        ph.fy = walk_frac(f0y, W.sfy, W.ry, wy, A.G.idy, tc);
        ph.fz = walk_frac(f0z, W.sfz, W.rz, wz, A.G.idz, tc);
        ph.ix = W.ix;
        ph.iy = W.iy;
        ph.iz = W.iz;
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
                                            int64_t& pix, int& local_pix, Real& vx, Real& vy, Real& vz, Real& r,
                                            Real& pre) {
    // X - X_c from voxel-local parts: the integer differences are exact
    const Real dx = ((Real)(ix - cam.icx) + (fx - cam.fcx)) * A.G.dx;
    const Real dy = ((Real)(iy - cam.icy) + (fy - cam.fcy)) * A.G.dy;
    const Real dz = ((Real)(iz - cam.icz) + (fz - cam.fcz)) * A.G.dz;
    const Real qz = cam.R[6] * dx + cam.R[7] * dy + cam.R[8] * dz;
    if (!(qz > (Real)0)) return false;
    const Real qx = cam.R[0] * dx + cam.R[1] * dy + cam.R[2] * dz;
    const Real qy = cam.R[3] * dx + cam.R[4] * dy + cam.R[5] * dz;
    const Real u = cam.fx * qx / qz + cam.cx;
    const Real v = cam.fy * qy / qz + cam.cy;
    if (!(u >= (Real)0 && u < cam.fw && v >= (Real)0 && v < cam.fh)) return false;
    const Real r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < (Real)1e-12) return false;
    local_pix = (int)v * cam.width + (int)u;
    pix = (int64_t)cam.pix_off + local_pix;
    r = m_sqrt(r2);
    const Real ir = (Real)1 / r;
    vx = -dx * ir;
    vy = -dy * ir;
    vz = -dz * ir;
    const Real cosang = wx * vx + wy * vy + wz * vz;
    pre = A.albedo * weight * hg_phase(A.g, cosang) / r2;
    return true;
}

// Steps (v)-(vi) after collision s: returns -1 while the photon lives, else
// its fate (capped or ended by Russian roulette).
template <typename Real>
__device__ __forceinline__ int after_collision(const KArgs<Real>& A, Photon<Real>& ph) {
    if (ph.s >= A.max_events) return MC_FATE_CAP;
    const uint4 r = draw(A.seed, ph.pid, ph.s);
    ph.weight *= A.albedo;
    if (ph.weight < A.rr) {
        if (uniform01<Real>(r.z) < ph.weight / A.rr) {
            ph.weight = A.rr;
        } else {
            return MC_FATE_RR;
        }
    }
    const Real omm = hg_one_minus_mu(A.g, uniform01<Real>(r.x));
    scatter_direction(ph.wx, ph.wy, ph.wz, omm, uniform01<Real>(r.y));
    ph.taustar = -m_log((Real)1 - uniform01<Real>(r.w));
    return -1;
}

// ---------------------------------------------------------------------------
// Local-estimate jobs.

// LDS queue of one wavefront (structure of arrays, ring of QCAP entries).
template <typename Real>
struct JobQueue {
    uint32_t vox[QCAP];  // start voxel packed as ix | iy << 11 | iz << 22
    Real fx[QCAP], fy[QCAP], fz[QCAP];
    Real vx[QCAP], vy[QCAP], vz[QCAP];
    Real r[QCAP], pre[QCAP];
    int32_t pix[QCAP];
};

// One lane's connection ray in flight.  The optical depth of a voxel is
// added one step after the walk entered it, so that the fetch of its
// extinction has a whole step to arrive: bn is in flight for the current
// voxel, (bp, lp) is the previous voxel's pending term.
template <typename Real>
struct Job {
    WalkRegs<Real> W;
    Real r;        // length to the camera
    Real bn, bp, lp;
    Real pre;      // albedo * I_s * P / r^2
    double tau;    // optical depth so far (FP64)
    double a;      // gradient weight of the second walk
    int pix;
    int phase;     // 1: optical depth, 2: gradient scatter
    uint32_t steps;
    // start of the ray, kept for the second walk of the gradient
    int i0x, i0y, i0z;
    Real f0x, f0y, f0z, vx, vy, vz;
};

template <typename Real>
__device__ __forceinline__ void job_begin(const KArgs<Real>& A, const uint32_t* mask, Job<Real>& J) {
    if (!walk_begin(J.W, A.G, J.i0x, J.i0y, J.i0z, J.f0x, J.f0y, J.f0z, J.vx, J.vy, J.vz)) {
        // cannot start: the first step ends the walk with zero length
        J.r = (Real)0;
        J.W.tx = J.W.ty = J.W.tz = (Real)0;
    }
    J.bn = J.phase == 2 ? (Real)0 : beta_at(A, mask, J.W);
    J.bp = (Real)0;
    J.lp = (Real)0;
    J.tau = 0.0;
    J.steps = 0;
}

// One voxel of the connection ray; returns true when the ray is done.
template <typename Real, int MODE, int TALLY>
__device__ __forceinline__ bool job_step(const KArgs<Real>& A, const uint32_t* mask, double* lds_grad, Job<Real>& J) {
    bool cx, cy, cz;
    const Real tn = walk_next(J.W, cx, cy, cz);
    const bool last = tn >= J.r;
    const Real tend = last ? J.r : tn;
    const Real l = tend - J.W.t;
    const bool scatter = MODE == MODE_GRAD && J.phase == 2;
    if (scatter) {
        grad_add<Real, TALLY>(A, lds_grad, J.W.k, -J.a * (double)l);
    } else {
        J.tau += (double)J.bp * (double)J.lp;
        J.bp = J.bn;
        J.lp = l;
        ++J.steps;
    }
    const bool out = walk_cross(J.W, A.G, tn, cx, cy, cz);
    const bool done = last || out;
    if (done) {
        if (!scatter) J.tau += (double)J.bp * (double)J.lp;
    } else if (!scatter) {
        J.bn = beta_at(A, mask, J.W);
    }
    return done;
}

// Tally of a finished ray.  For the gradient, a finished first walk with a
// non-zero weight starts the second walk (returns true: the lane stays busy).
//
// With the tape, a ray with a non-zero weight instead starts a walk over the
// grid of tiles (emit: its records are written by emit_records).
template <typename Real, int MODE, int TALLY>
__device__ __forceinline__ bool job_finish(const KArgs<Real>& A, const uint32_t* mask, double* lds_grad, Job<Real>& J,
                                           uint64_t& vconn, bool& emit) {
    if (MODE == MODE_GRAD && J.phase == 2) return false;
    vconn += J.steps;
    const double C = (double)J.pre * (double)m_exp((Real)(-J.tau));
    if (MODE == MODE_RENDER) {
        tally_f64<TALLY>(A.img, A.img32, J.pix, C);
        if (A.img_m2) unsafeAtomicAdd(A.img_m2 + J.pix, C * C);
        return false;
    } else {
        const double a = A.gw[J.pix] * C;
        if (a == 0.0) return false;
        if (A.tape) {
            const Tape<Real>& P = A.tp;
            const int tix = J.i0x / P.tx, tiy = J.i0y / P.ty, tiz = J.i0z / P.tz;
            const Real ftx = ((Real)(J.i0x - tix * P.tx) + J.f0x) * P.itx;
            const Real fty = ((Real)(J.i0y - tiy * P.ty) + J.f0y) * P.ity;
            const Real ftz = ((Real)(J.i0z - tiz * P.tz) + J.f0z) * P.itz;
            if (!walk_begin(J.W, P.T, tix, tiy, tiz, ftx, fty, ftz, J.vx, J.vy, J.vz)) {
                // only the start tile
                J.W.tx = J.W.ty = J.W.tz = (Real)INFINITY;
            }
            J.a = a;
            emit = true;
            return false;
        }
        const int ke = J.i0x + A.G.nx * J.i0y + A.G.nxy * J.i0z;
        grad_add<Real, TALLY>(A, lds_grad, ke, a / (double)A.beta[ke]);
        J.a = a;
        J.phase = 2;
        job_begin(A, mask, J);
        return true;
    }
}

// Tape records of the rays whose lanes have `emit` set: one record per lane
// and step, for the tile the lane's tile walk is in, then the walk moves to
// the next tile.  Slots are handed out per wavefront: `tab` (LDS, private to
// the wavefront) holds for every tile the base, the used count and the size
// of the block of slots the wavefront reserved last.  Appends take positions
// with LDS atomics; the first lane past the end of a block reserves the next
// one from the tile's device counter (one device atomic per block, not per
// record).  A reservation beyond the tile's capacity sets the overflow flag
// and its records are dropped (the host then replays the chunk smaller).
template <typename Real>
__device__ __forceinline__ void emit_records(const KArgs<Real>& A, uint32_t* tab, Job<Real>& J, bool& emit) {
    const Tape<Real>& P = A.tp;
    uint32_t* t_base = tab;
    uint32_t* t_used = tab + P.n_tiles;
    uint32_t* t_size = tab + 2 * P.n_tiles;
    while (__ballot(emit)) {
        const int t = emit ? J.W.k : 0;
        uint32_t pos = 0, base = 0, size = 0;
        if (emit) {
            pos = atomicAdd(&t_used[t], 1u);
            base = t_base[t];
            size = t_size[t];
        }
        const bool spill = emit && pos >= size;
        if (__ballot(spill)) {
            if (spill && pos == size) {
                // positions of one tile are consecutive from the used count,
                // which never exceeds the size: exactly one lane per tile
                // lands on the end of the block
                const uint32_t n_sp = t_used[t] - size;
                const uint32_t need = n_sp > P.block ? n_sp : P.block;
                const uint32_t nb = atomicAdd(&P.count[t], need);
                if ((uint64_t)nb + need > (uint64_t)P.cap[t]) P.overflow[0] = 1u;
                t_base[t] = nb;
                t_used[t] = n_sp;
                t_size[t] = need;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            if (spill) {
                base = t_base[t];
                pos -= size;
            }
        }
        if (emit) {
            const uint32_t slot = base + pos;
            if (slot < P.cap[t]) {
                const uint32_t i = P.off[t] + slot;
                P.vox[i] = (uint32_t)J.i0x | ((uint32_t)J.i0y << 11) | ((uint32_t)J.i0z << 22);
                P.fx[i] = J.f0x;
                P.fy[i] = J.f0y;
                P.fz[i] = J.f0z;
                P.vx[i] = J.vx;
                P.vy[i] = J.vy;
                P.vz[i] = J.vz;
                P.r[i] = J.r;
                P.a[i] = (Real)J.a;
            }
            bool cx, cy, cz;
            const Real tn = walk_next(J.W, cx, cy, cz);
            if (tn >= J.r || walk_cross(J.W, P.T, tn, cx, cy, cz)) emit = false;
        }
    }
}

// Job phase of one wavefront.  Not final: return once fewer jobs are queued
// or in flight than there are lanes.  Final: run until everything is done.
template <typename Real, int MODE, int TALLY>
__device__ __forceinline__ void drain(const KArgs<Real>& A, const uint32_t* mask, double* lds_grad, uint32_t* tab,
                                      JobQueue<Real>& Q, uint32_t& qhead, uint32_t qtail, Job<Real>& J, bool& busy,
                                      bool& fin, bool final_pass, uint64_t& vconn) {
    for (;;) {
        bool emit = false;
        if (fin) {
            fin = false;
            busy = job_finish<Real, MODE, TALLY>(A, mask, lds_grad, J, vconn, emit);
        }
        if (MODE == MODE_GRAD && A.tape) emit_records(A, tab, J, emit);
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
                    J.phase = 1;
                    job_begin(A, mask, J);
                    busy = true;
                }
            }
            qhead += take;
        }
        // walk until a quarter of the lanes are idle (all, if nothing is queued)
        const uint32_t keep = (qtail - qhead) > 0 ? (uint32_t)WAVE - REFILL_IDLE : 0u;
        while ((uint32_t)__popcll(__ballot(busy)) > keep) {
            if (busy && job_step<Real, MODE, TALLY>(A, mask, lds_grad, J)) {
                busy = false;
                fin = true;
            }
        }
    }
}

// Dynamic LDS of k_render: the occupancy bitmask (mask_words), then, when
// the gradient is privatised, one double per voxel, or with the tape, every
// wavefront's slot table (3 words per tile).
template <typename Real, int MODE, int TALLY>
__global__ void __launch_bounds__(BLOCK) k_render(KArgs<Real> A) {
    __shared__ JobQueue<Real> s_q[WAVES];
    __shared__ unsigned long long s_st[ST_N];
    extern __shared__ uint32_t s_dyn[];
    uint32_t* s_mask = s_dyn;
    double* lds_grad = nullptr;
    uint32_t* tab = nullptr;
    if (MODE == MODE_GRAD && A.grad_lds) {
        lds_grad = reinterpret_cast<double*>(s_dyn + ((A.mask_words + 1) & ~1));
        for (int64_t i = threadIdx.x; i < A.n_vox; i += BLOCK) lds_grad[i] = 0.0;
    }
    if (MODE == MODE_GRAD && A.tape) {
        uint32_t* all = s_dyn + ((A.mask_words + 1) & ~1);
        // used = size = 0: the first append to a tile reserves a block
        for (int i = threadIdx.x; i < WAVES * 3 * A.tp.n_tiles; i += BLOCK) all[i] = 0u;
        tab = all + (threadIdx.x / WAVE) * 3 * A.tp.n_tiles;
    }
    if (threadIdx.x < ST_N) s_st[threadIdx.x] = 0ull;
    for (int i = threadIdx.x; i < A.mask_words; i += BLOCK) s_mask[i] = A.mask[i];
    __syncthreads();
    const uint32_t* mask = s_mask;
    JobQueue<Real>& Q = s_q[threadIdx.x / WAVE];

    Photon<Real> ph;
    Job<Real> J;
    bool alive = false, exhausted = false, busy = false, fin = false;
    uint32_t qhead = 0, qtail = 0;
    uint32_t n_ev = 0, n_le = 0;
    uint64_t vfree = 0, vconn = 0;

    for (;;) {
        if (!alive && !exhausted) {
            const uint64_t k = wave_fetch(A.work);
            if (k < A.n_photons) {
                launch_photon(A, A.pid0 + k, ph);
                alive = true;
            } else {
                exhausted = true;
            }
        }
        if (__ballot(alive) == 0ull) break;
        bool collided = false;
        if (alive) {
            const int left = free_flight(A, mask, ph, vfree);
            if (left) {
                atomicAdd(&s_st[ST_TOP + left - 1], 1ull);
                alive = false;
            } else {
                collided = true;
                ph.s += 1;
                ++n_ev;
            }
        }
        if (__ballot(collided)) {
            for (int c = 0; c < A.n_cams; ++c) {
                const DevCam<Real>& cam = A.cams[c];
                int64_t pix = 0;
                int lp = 0;
                Real vx = 0, vy = 0, vz = 0, r = 0, pre = 0;
                const bool vis = collided && le_geometry(A, cam, ph.ix, ph.iy, ph.iz, ph.fx, ph.fy, ph.fz, ph.wx,
                                                         ph.wy, ph.wz, ph.weight, pix, lp, vx, vy, vz, r, pre);
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
                    Q.pre[slot] = pre;
                    Q.pix[slot] = (int32_t)pix;
                    ++n_le;
                }
                qtail += (uint32_t)__popcll(m);
                if (qtail - qhead > QCAP - (uint32_t)WAVE)
                    drain<Real, MODE, TALLY>(A, mask, lds_grad, tab, Q, qhead, qtail, J, busy, fin, false, vconn);
            }
        }
        if (collided) {
            const int fate = after_collision(A, ph);
            if (fate >= 0) {
                atomicAdd(&s_st[fate == MC_FATE_CAP ? ST_CAP : ST_RR], 1ull);
                alive = false;
            }
        }
        drain<Real, MODE, TALLY>(A, mask, lds_grad, tab, Q, qhead, qtail, J, busy, fin, false, vconn);
    }
    drain<Real, MODE, TALLY>(A, mask, lds_grad, tab, Q, qhead, qtail, J, busy, fin, true, vconn);

    if (n_ev) atomicAdd(&s_st[ST_EVENTS], (unsigned long long)n_ev);
    if (n_le) atomicAdd(&s_st[ST_LE], (unsigned long long)n_le);
    if (vfree) atomicAdd(&s_st[ST_VFREE], (unsigned long long)vfree);
    if (vconn) atomicAdd(&s_st[ST_VCONN], (unsigned long long)vconn);
    __syncthreads();
    if (threadIdx.x < ST_N && s_st[threadIdx.x]) atomicAdd(&A.stats[threadIdx.x], s_st[threadIdx.x]);
    if (lds_grad) {
        for (int64_t i = threadIdx.x; i < A.n_vox; i += BLOCK) {
            const double v = lds_grad[i];
            if (v != 0.0) tally_f64<TALLY>(A.grad, A.grad32, i, v);
        }
    }
}

// ---------------------------------------------------------------------------
// Gradient deposit of one tile: the block accumulates in LDS, for the tape
// slots [lo, hi) of its tile, -a l(m) along every recorded ray inside the
// tile and a / beta(k_e) for the rays that start in it, then adds the tile
// to the gradient (one device atomic per touched voxel).

// Start the walk of the tape record in slot i (tile-local coordinates; the
// walk's linear index is the LDS index).  False when the record is empty or
// the ray has no length inside the tile.
template <typename Real>
__device__ __forceinline__ bool deposit_begin(const KArgs<Real>& A, const DevGrid<Real>& L, int b0x, int b0y, int b0z,
                                              uint32_t i, double* s_g, WalkRegs<Real>& W, Real& len, double& a) {
    const Tape<Real>& P = A.tp;
    const Real ar = P.a[i];
    if (ar == (Real)0) return false;
    a = (double)ar;
    const uint32_t v = P.vox[i];
    const int i0x = (int)(v & 2047u), i0y = (int)((v >> 11) & 2047u), i0z = (int)(v >> 22);
    const Real f0x = P.fx[i], f0y = P.fy[i], f0z = P.fz[i];
    const Real vx = P.vx[i], vy = P.vy[i], vz = P.vz[i];
    const Real r = P.r[i];
    const int jx = i0x - b0x, jy = i0y - b0y, jz = i0z - b0z;
    if ((unsigned)jx < (unsigned)L.nx && (unsigned)jy < (unsigned)L.ny && (unsigned)jz < (unsigned)L.nz) {
        const int ke = i0x + A.G.nx * i0y + A.G.nxy * i0z;
        atomicAdd(s_g + (jx + L.nx * jy + L.nxy * jz), a / (double)A.beta[ke]);
    }
    // clip [0, r] to the tile box, in tile-local voxel units (double)
    const double o[3] = {(double)jx + (double)f0x, (double)jy + (double)f0y, (double)jz + (double)f0z};
    const double u[3] = {(double)vx / (double)L.dx, (double)vy / (double)L.dy, (double)vz / (double)L.dz};
    const int e[3] = {L.nx, L.ny, L.nz};
    double t0 = 0.0, t1 = (double)r;
    for (int ax = 0; ax < 3; ++ax) {
        if (u[ax] > 1e-300 || u[ax] < -1e-300) {
            const double ta = (0.0 - o[ax]) / u[ax], tb = ((double)e[ax] - o[ax]) / u[ax];
            t0 = fmax(t0, fmin(ta, tb));
            t1 = fmin(t1, fmax(ta, tb));
        } else if (!(o[ax] >= 0.0 && o[ax] <= (double)e[ax])) {
            return false;
        }
    }
    if (!(t1 > t0)) return false;
    int j[3];
    Real f[3];
    for (int ax = 0; ax < 3; ++ax) {
        const double p = o[ax] + t0 * u[ax];
        double fl = floor(p);
        fl = fl < 0.0 ? 0.0 : (fl > (double)(e[ax] - 1) ? (double)(e[ax] - 1) : fl);
        double fr = p - fl;
        fr = fr < 0.0 ? 0.0 : (fr > 1.0 ? 1.0 : fr);
        j[ax] = (int)fl;
        f[ax] = (Real)fr;
    }
    if (!walk_begin(W, L, j[0], j[1], j[2], f[0], f[1], f[2], vx, vy, vz)) return false;
    len = (Real)(t1 - t0);
    return true;
}

template <typename Real, int TALLY>
__global__ void __launch_bounds__(DEPOSIT_BLOCK) k_deposit(KArgs<Real> A, const DepositItem* items) {
    __shared__ double s_g[TILE_VOX];
    __shared__ uint32_t s_next;
    const Tape<Real>& P = A.tp;
    const DepositItem it = items[blockIdx.x];
    const int tix = it.tile % P.T.nx, tiy = (it.tile / P.T.nx) % P.T.ny, tiz = it.tile / P.T.nxy;
    const int b0x = tix * P.tx, b0y = tiy * P.ty, b0z = tiz * P.tz;
    DevGrid<Real> L = A.G;
    L.nx = min(P.tx, A.G.nx - b0x);
    L.ny = min(P.ty, A.G.ny - b0y);
    L.nz = min(P.tz, A.G.nz - b0z);
    L.nxy = L.nx * L.ny;
    const int nloc = L.nxy * L.nz;
    for (int i = threadIdx.x; i < nloc; i += DEPOSIT_BLOCK) s_g[i] = 0.0;
    if (threadIdx.x == 0) s_next = it.lo;
    __syncthreads();

    const uint32_t base = P.off[it.tile];
    WalkRegs<Real> W;
    Real len = (Real)0;
    double a = 0.0;
    bool busy = false, more = true;
    for (;;) {
        if (more) {
            // idle lanes take the next slots of the block's range
            const unsigned long long idle = __ballot(!busy);
            if (idle) {
                const int leader = __ffsll((long long)idle) - 1;
                uint32_t first = 0;
                if (__lane_id() == leader) first = atomicAdd(&s_next, (uint32_t)__popcll(idle));
                first = __shfl(first, leader);
                if (first >= it.hi) more = false;
                if (!busy) {
                    const uint32_t s = first + lanes_below(idle);
                    if (s < it.hi) busy = deposit_begin(A, L, b0x, b0y, b0z, base + s, s_g, W, len, a);
                }
            }
        }
        if (!more && __ballot(busy) == 0ull) break;
        const uint32_t keep = more ? (uint32_t)WAVE - REFILL_IDLE : 0u;
        while ((uint32_t)__popcll(__ballot(busy)) > keep) {
            if (busy) {
                bool cx, cy, cz;
                const Real tn = walk_next(W, cx, cy, cz);
                const bool last = tn >= len;
                const Real l = (last ? len : tn) - W.t;
                atomicAdd(s_g + W.k, -a * (double)l);
                if (walk_cross(W, L, tn, cx, cy, cz) || last) busy = false;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nloc; i += DEPOSIT_BLOCK) {
        const double v = s_g[i];
        if (v != 0.0) {
            const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / L.nxy;
            tally_f64<TALLY>(A.grad, A.grad32, (int64_t)(b0x + x) + (int64_t)A.G.nx * (b0y + y) +
                                                   (int64_t)A.G.nxy * (b0z + z), v);
        }
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
        const int left = free_flight(A, (const uint32_t*)nullptr, ph, vfree);
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
                                             ph.wz, ph.weight, pix, lp, vx, vy, vz, r, pre);
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
    for (int j = 0; j < 9; ++j) d.R[j] = (Real)h.R[j];
    d.fx = (Real)h.fx;
    d.fy = (Real)h.fy;
    d.cx = (Real)h.cx;
    d.cy = (Real)h.cy;
    d.fw = (Real)h.width;
    d.fh = (Real)h.height;
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
// set when cell 32 w + j holds a voxel with beta > 0 (or a non-finite beta,
// which must reach the walk unchanged).
template <typename Real>
__global__ void k_build_mask(KArgs<Real> A, uint32_t* mask, int ncz) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= A.mask_words) return;
    const int64_t ncells = (int64_t)A.mncx * A.mncy * ncz;
    uint32_t word = 0;
    for (int j = 0; j < 32; ++j) {
        const int64_t cell = (int64_t)w * 32 + j;
        if (cell >= ncells) break;
        const int cx = (int)(cell % A.mncx), cy = (int)((cell / A.mncx) % A.mncy), cz = (int)(cell / ((int64_t)A.mncx * A.mncy));
        const int x0 = cx << A.mshx, y0 = cy << A.mshy, z0 = cz << A.mshz;
        const int x1 = min(x0 + (1 << A.mshx), A.G.nx), y1 = min(y0 + (1 << A.mshy), A.G.ny),
                  z1 = min(z0 + (1 << A.mshz), A.G.nz);
        bool any = false;
        for (int z = z0; z < z1 && !any; ++z)
            for (int y = y0; y < y1 && !any; ++y)
                for (int x = x0; x < x1 && !any; ++x) {
                    const Real b = A.beta[x + A.G.nx * y + A.G.nxy * z];
                    any = !(b == (Real)0);
                }
        if (any) word |= 1u << j;
    }
    mask[w] = word;
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
    if (mode == MODE_GRAD && a.tape) bytes += (size_t)WAVES * 3 * a.tp.n_tiles * sizeof(uint32_t);
    return bytes;
}

template <typename Real, int MODE, int TALLY>
static hipError_t launch_r(const KArgs<Real>& a, int grid, hipStream_t s) {
    const size_t dyn = render_dyn_lds(a, MODE);
    hipLaunchKernelGGL((k_render<Real, MODE, TALLY>), dim3(grid), dim3(BLOCK), dyn, s, a);
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_transport(const KArgs<Real>& a, int mode, int tally, int grid, hipStream_t s) {
    if (mode == MODE_RENDER) {
        return tally == TALLY_F64 ? launch_r<Real, MODE_RENDER, TALLY_F64>(a, grid, s)
                                  : launch_r<Real, MODE_RENDER, TALLY_K32>(a, grid, s);
    }
    if (mode == MODE_GRAD) {
        return tally == TALLY_F64 ? launch_r<Real, MODE_GRAD, TALLY_F64>(a, grid, s)
                                  : launch_r<Real, MODE_GRAD, TALLY_K32>(a, grid, s);
    }
    hipLaunchKernelGGL(k_trace<Real>, dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <typename Real, int MODE, int TALLY>
static hipError_t occ_r(const KArgs<Real>& a, int* b) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(b, (const void*)k_render<Real, MODE, TALLY>, BLOCK,
                                                        render_dyn_lds(a, MODE));
}

template <typename Real>
hipError_t transport_occupancy(const KArgs<Real>& a, int mode, int tally, int* b) {
    if (mode == MODE_RENDER) return tally == TALLY_F64 ? occ_r<Real, MODE_RENDER, TALLY_F64>(a, b)
                                                       : occ_r<Real, MODE_RENDER, TALLY_K32>(a, b);
    if (mode == MODE_GRAD) return tally == TALLY_F64 ? occ_r<Real, MODE_GRAD, TALLY_F64>(a, b)
                                                     : occ_r<Real, MODE_GRAD, TALLY_K32>(a, b);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(b, (const void*)k_trace<Real>, BLOCK, 0);
}

template <typename Real>
hipError_t launch_build_mask(const KArgs<Real>& a, uint32_t* mask, int ncz, hipStream_t s) {
    hipLaunchKernelGGL(k_build_mask<Real>, dim3(blocks_for(a.mask_words)), dim3(BLOCK), 0, s, a, mask, ncz);
    return hipGetLastError();
}

template <typename Real>
hipError_t launch_deposit(const KArgs<Real>& a, int tally, const DepositItem* items, int n_items, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (tally == TALLY_F64)
        hipLaunchKernelGGL((k_deposit<Real, TALLY_F64>), dim3(n_items), dim3(DEPOSIT_BLOCK), 0, s, a, items);
    else
        hipLaunchKernelGGL((k_deposit<Real, TALLY_K32>), dim3(n_items), dim3(DEPOSIT_BLOCK), 0, s, a, items);
    return hipGetLastError();
}

template hipError_t launch_deposit<float>(const KArgs<float>&, int, const DepositItem*, int, hipStream_t);
template hipError_t launch_deposit<double>(const KArgs<double>&, int, const DepositItem*, int, hipStream_t);
template hipError_t launch_build_mask<float>(const KArgs<float>&, uint32_t*, int, hipStream_t);
template hipError_t launch_build_mask<double>(const KArgs<double>&, uint32_t*, int, hipStream_t);
template hipError_t launch_write_cams<float>(const CamChunk&, DevCam<float>*, NormCam*, hipStream_t);
template hipError_t launch_write_cams<double>(const CamChunk&, DevCam<double>*, NormCam*, hipStream_t);
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
