// Device building blocks of the gfx950 renderer: counter-based random
// numbers, Henyey-Greenstein phase function and sampling, the scattering
// frame, pinhole projection and the voxel walk.
//
// Method: Holodovsky et al., "In-situ multi-scattering tomography"
// (arXiv 1512.02110), Sec. 2.1 and Sec. 3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcrt {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32 -> 64-bit products with the published multipliers; the key advances
// by the published Weyl increments between rounds.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

// Uniform in (0,1) on a 2^23 grid, exactly representable in FP32 and FP64.
template <typename Real>
__device__ __forceinline__ Real uniform01(uint32_t x) {
    return (Real)((float)(x >> 9) + 0.5f) * (Real)(1.0f / 8388608.0f);
}

// Leg `leg` of photon `pid`: counter (pid lo, pid hi, leg, 0), key = seed.
__device__ __forceinline__ uint4 draw(uint64_t seed, uint64_t pid, uint32_t leg) {
    return philox4x32_10(make_uint4((uint32_t)pid, (uint32_t)(pid >> 32), leg, 0u),
                         make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
}

// ---------------------------------------------------------------------------
// Precision-dependent math.
// The FP64 log and sincospi (the photon's free path and scattering azimuth)
// are called, not inlined: inlined, the compiler keeps their polynomial
// coefficients in VGPR pairs for the whole kernel (a 64-bit constant is no
// inline operand) and the mixed-precision render, held to 128 VGPRs, spills
// them to scratch and reloads them in its main loop.  Called, they use
// registers only inside the call (the same results; the mixed render 6%
// faster, the FP64 render unchanged).
__device__ __forceinline__ float m_log(float x) { return logf(x); }
__device__ __attribute__((noinline)) double m_log(double x) { return log(x); }
__device__ __forceinline__ float m_exp(float x) { return expf(x); }
__device__ __forceinline__ double m_exp(double x) { return exp(x); }
__device__ __forceinline__ float m_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double m_sqrt(double x) { return sqrt(x); }
// Square root without the IEEE refinement (float: the hardware's ~1 ulp
// result); for lengths whose last bit does not matter.
__device__ __forceinline__ float m_sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double m_sqrt_fast(double x) { return sqrt(x); }
__device__ __forceinline__ float m_rsqrt(float x) { return 1.0f / sqrtf(x); }
__device__ __forceinline__ double m_rsqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float m_cbrt(float x) { return cbrtf(x); }
__device__ __forceinline__ double m_cbrt(double x) { return cbrt(x); }
__device__ __forceinline__ float m_floor(float x) { return floorf(x); }
__device__ __forceinline__ double m_floor(double x) { return floor(x); }
__device__ __forceinline__ void m_sincospi(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __attribute__((noinline)) void m_sincospi(double x, double* s, double* c) { sincospi(x, s, c); }
// reciprocal: one hardware instruction (about 1 ulp) in FP32, exact division in FP64
__device__ __forceinline__ float m_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double m_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float m_fma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double m_fma(double a, double b, double c) { return fma(a, b, c); }

// Rayleigh phase function, Eq. (Pray): 3 (1 + cos^2) / (16 pi).
template <typename Real>
__device__ __forceinline__ Real rayleigh_phase(Real cosang) {
    return (Real)0.05968310365946075 * ((Real)1 + cosang * cosang);
}

// Inverse-transform sample of the Rayleigh polar cosine, Eq. (thetaREY):
// mu = c - 1/c, c the cube root of gamma = 4u - 2 + sqrt((4u - 2)^2 + 1)
// (the real root of (mu^3 + 3 mu + 4) / 8 = u).  Returns 1 - mu.
template <typename Real>
__device__ __forceinline__ Real rayleigh_one_minus_mu(Real u) {
    const Real a = (Real)4 * u - (Real)2;
    const Real c = m_cbrt(a + m_sqrt(a * a + (Real)1));
    Real omm = (Real)1 - (c - (Real)1 / c);
    omm = omm < (Real)0 ? (Real)0 : omm;
    return omm > (Real)2 ? (Real)2 : omm;
}

// Henyey-Greenstein phase function, Eq. (Phg), as a function of the cosine
// of the scattering angle.
template <typename Real>
__device__ __forceinline__ Real hg_phase(Real g, Real cosang) {
    const Real den = (Real)1 + g * g - (Real)2 * g * cosang;
    return ((Real)1 - g * g) * (Real)0.07957747154594767 / (den * m_sqrt(den));
}

// Inverse-transform sample of the HG polar cosine (Eq. thetaHG with the
// square restored), written as 1 - mu = (1-g)(1-u)(s+1-g)/(1-g+2gu),
// s = (1-g^2)/(1-g+2gu): no cancellation near mu = 1 and exact at g = 0.
// Returns 1 - mu (in [0, 2]).
template <typename Real>
__device__ __forceinline__ Real hg_one_minus_mu(Real g, Real u) {
    const Real a = (Real)1 - g + (Real)2 * g * u;
    const Real s = ((Real)1 - g * g) / a;
    Real omm = ((Real)1 - g) * ((Real)1 - u) * (s + (Real)1 - g) / a;
    omm = omm < (Real)0 ? (Real)0 : omm;
    return omm > (Real)2 ? (Real)2 : omm;
}

// New unit direction at polar cosine mu (given as 1 - mu) and azimuth
// 2 pi u about w, on the orthonormal basis of Duff et al. (JCGT 2017),
// renormalised.
template <typename Real>
__device__ __forceinline__ void scatter_direction(Real& wx, Real& wy, Real& wz, Real omm, Real u_phi) {
    const Real mu = (Real)1 - omm;
    const Real st = m_sqrt(omm * ((Real)2 - omm));  // sin = sqrt((1-mu)(1+mu))
    Real sp, cp;
    m_sincospi((Real)2 * u_phi, &sp, &cp);
    const Real sign = wz >= (Real)0 ? (Real)1 : (Real)-1;
    const Real a = (Real)-1 / (sign + wz);
    const Real b = wx * wy * a;
    const Real b1x = (Real)1 + sign * wx * wx * a, b1y = sign * b, b1z = -sign * wx;
    const Real b2x = b, b2y = sign + wy * wy * a, b2z = -wy;
    const Real c1 = st * cp, c2 = st * sp;
    Real nx = c1 * b1x + c2 * b2x + mu * wx;
    Real ny = c1 * b1y + c2 * b2y + mu * wy;
    Real nz = c1 * b1z + c2 * b2z + mu * wz;
    const Real inv = m_rsqrt(nx * nx + ny * ny + nz * nz);
    wx = nx * inv;
    wy = ny * inv;
    wz = nz * inv;
}

// ---------------------------------------------------------------------------
// Grid and camera tables as the kernels see them.
//
// Positions are kept voxel-local: an integer voxel (ix, iy, iz) and the
// fraction (fx, fy, fz) in [0, 1] of the voxel edge along each axis.  The
// rounding error of a position is then relative to the voxel edge, not to
// the domain size, which keeps FP32 transport close to FP64 in thick cloud
// (short flights) and makes the projection of collisions close to a camera
// accurate relative to their distance.
template <typename Real>
struct DevGrid {
    int nx, ny, nz, nxy;
    Real dx, dy, dz;     // voxel edges (km)
    Real idx, idy, idz;  // 1 / edge
    double ddx, ddy, ddz;  // voxel edges in double (the projection onto the cameras)
};

// A camera as the kernels see it.  The connection rays use the centre in the
// transport precision; the projection of a collision (its pixel and the cull
// of collisions at the centre) is computed in FP64 whatever the transport
// precision, from the camera's double parameters, so that the pixel of a
// local estimate depends only on the collision point the transport computed
// and not on the rounding of the projection.
template <typename Real>
struct DevCam {
    int32_t icx, icy, icz;  // camera centre = (ic + fc) voxel edges along each axis
    int32_t width;
    Real fcx, fcy, fcz;
    int32_t pix_off, pad_;
    double pfcx, pfcy, pfcz;  // the centre's fraction in double
    double R[9];
    double fx, fy, cx, cy;
    double fw, fh;  // width, height
};

// Voxel walk (regular tracking) from the voxel-local point (i, f) along the
// unit direction w.  The ray parameter t is a length in km.  The next face
// crossing on axis a is t_a = (m_a - f_a) * d_a / w_a with m_a the index of
// that face counted from the start voxel's lower face, recomputed after each
// crossing (no accumulated error).  Ties between axes go to the lowest axis.
//
// The kernels keep the walk state in plain local scalars so that every
// per-axis choice is a register select (a choice between members of a struct
// lets the compiler select between their addresses instead, which sends the
// walk state to scratch memory).
template <typename Real>
struct WalkAxis {
    // Direction components below `tiny` count as zero, so that every axis
    // with a non-zero step has a finite crossing parameter.
    static constexpr Real tiny = sizeof(Real) == 4 ? (Real)1e-20f : (Real)1e-200;

    __device__ __forceinline__ static void init(Real f, Real w, Real d, int& s, Real& m, Real& tn, Real& g) {
        s = w > tiny ? 1 : (w < -tiny ? -1 : 0);
        if (s != 0) {
            g = d / w;
            m = s > 0 ? (Real)1 : (Real)0;
            tn = (m - f) * g;
            tn = tn < (Real)0 ? (Real)0 : tn;
        } else {
            g = (Real)0;
            m = (Real)0;
            tn = (Real)INFINITY;
        }
    }

    // Fraction along one axis of the point at parameter tp, relative to the
    // current voxel (after the walk's crossings on that axis), clamped to [0, 1].
    __device__ __forceinline__ static Real frac_at(Real f0, int s, Real m, Real w, Real id, Real tp) {
        const Real crossed = m - (s > 0 ? (Real)1 : (Real)0);
        Real q = f0 + tp * w * id - crossed;
        q = q < (Real)0 ? (Real)0 : q;
        return q > (Real)1 ? (Real)1 : q;
    }
};

// Number of voxels a walk from (ax, ay, az) to (bx, by, bz) visited: one per
// crossing, plus the final voxel when the walk ended inside the domain.
__device__ __forceinline__ uint32_t walk_voxels(int ax, int ay, int az, int bx, int by, int bz, bool inside) {
    return (uint32_t)(abs(bx - ax) + abs(by - ay) + abs(bz - az)) + (inside ? 1u : 0u);
}

}  // namespace mcrt
