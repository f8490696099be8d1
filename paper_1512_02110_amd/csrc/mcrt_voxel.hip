// Voxelised forward model of Sec. 3, deterministic part, in FP64: the
// transmittance T_c(k) from every voxel centre to every camera (Eqs.
// taoKtoc, Tck), the images i_c = Pi_c (j_c . beta . T_c) with n x n
// sub-pixel rays (Eqs. IcP, PIc, Icpixel), and the gradient of a loss of
// those images with j frozen (Eqs. Jaco1, TcofJaco1, DivTc):
//   grad(m) = sum_c [ T_c(m) j_c(m) B_c(m)
//                     - sum_k D_c(k, m) T_c(k) beta(k) j_c(k) B_c(k) ],
// B_c = Pi_c^T dL/di_c, D_c(k, m) the length in voxel m of the line of sight
// from the centre of voxel k to camera c.
//
// One thread per line of sight (T, gradient) or per pixel (images,
// back-projection); each walks the voxels of its segment.  The images are
// gathers (no atomics); B and the gradient are scatters with device FP64
// atomics (at most a few times 1e8 per call for the benchmark grids).
#include <cmath>

#include "mcrt_internal.hpp"

namespace mcrt {
namespace {

constexpr int VOX_BLOCK = 256;

// Voxels of the segment p + t v, t in [0, tmax] (v unit), that lie in the
// domain, in order: f(k, length inside k).  The segment is clipped to the
// domain box first; a point on a face belongs to the voxel on the side the
// segment moves into; ties between axes go to the lowest axis.  Crossings
// are recomputed from the segment's start after every step (no accumulated
// rounding).
template <typename F>
__device__ void seg_walk(const VoxArgs& A, double px, double py, double pz, double vx, double vy, double vz,
                         double tmax, F&& f) {
    const double p[3] = {px, py, pz};
    const double v[3] = {vx, vy, vz};
    const double d[3] = {A.dx, A.dy, A.dz};
    const int n[3] = {A.nx, A.ny, A.nz};
    double t0 = 0.0, t1 = tmax;
    for (int a = 0; a < 3; ++a) {
        const double len = n[a] * d[a];
        if (v[a] == 0.0) {
            if (p[a] < 0.0 || p[a] > len) return;
            continue;
        }
        const double ta = (0.0 - p[a]) / v[a], tb = (len - p[a]) / v[a];
        t0 = fmax(t0, fmin(ta, tb));
        t1 = fmin(t1, fmax(ta, tb));
    }
    if (!(t1 > t0)) return;
    int idx[3], step[3];
    double tn[3];
    for (int a = 0; a < 3; ++a) {
        const double x = (p[a] + t0 * v[a]) / d[a];
        int i = (int)floor(x);
        if (v[a] < 0.0 && x == floor(x)) i -= 1;
        i = i < 0 ? 0 : (i > n[a] - 1 ? n[a] - 1 : i);
        idx[a] = i;
        step[a] = v[a] > 0.0 ? 1 : (v[a] < 0.0 ? -1 : 0);
        tn[a] = step[a] == 0 ? INFINITY : ((double)(i + (step[a] > 0 ? 1 : 0)) * d[a] - p[a]) / v[a];
    }
    const int64_t stride[3] = {1, (int64_t)A.nx, (int64_t)A.nx * A.ny};
    int64_t k = idx[0] + stride[1] * idx[1] + stride[2] * idx[2];
    double t = t0;
    for (;;) {
        int a = 0;
        if (tn[1] < tn[a]) a = 1;
        if (tn[2] < tn[a]) a = 2;
        const bool last = tn[a] >= t1;
        f(k, (last ? t1 : tn[a]) - t);
        if (last) return;
        t = tn[a];
        idx[a] += step[a];
        if (idx[a] < 0 || idx[a] >= n[a]) return;
        k += step[a] * stride[a];
        tn[a] = ((double)(idx[a] + (step[a] > 0 ? 1 : 0)) * d[a] - p[a]) / v[a];
    }
}

__device__ void voxel_centre(const VoxArgs& A, int64_t k, double& x, double& y, double& z) {
    const int64_t nxy = (int64_t)A.nx * A.ny;
    x = ((double)(k % A.nx) + 0.5) * A.dx;
    y = ((double)((k / A.nx) % A.ny) + 0.5) * A.dy;
    z = ((double)(k / nxy) + 0.5) * A.dz;
}

// Camera of global pixel p (the last camera whose first pixel is <= p).
__device__ int camera_of_pixel(const VoxArgs& A, int64_t p) {
    int lo = 0, hi = A.n_cams - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (A.cams[mid].pix_off <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Unit direction of sub-pixel ray (a, b) of pixel (row, col): through the
// image point (col + (a + 1/2)/n, row + (b + 1/2)/n), back-projected
// (world = R^T camera).
__device__ void subpixel_dir(const HostCam& c, int row, int col, int a, int b, int n, double& vx, double& vy,
                             double& vz) {
    const double qx = ((double)col + (a + 0.5) / n - c.cx) / c.fx;
    const double qy = ((double)row + (b + 0.5) / n - c.cy) / c.fy;
    vx = c.R[0] * qx + c.R[3] * qy + c.R[6];
    vy = c.R[1] * qx + c.R[4] * qy + c.R[7];
    vz = c.R[2] * qx + c.R[5] * qy + c.R[8];
    const double il = 1.0 / sqrt(vx * vx + vy * vy + vz * vz);
    vx *= il;
    vy *= il;
    vz *= il;
}

__global__ void k_vox_cams(CamChunk chunk, HostCam* dev) {
    const int i = threadIdx.x;
    if (i < chunk.n) dev[chunk.first + i] = chunk.c[i];
}

// T_c(k) for every camera and voxel (Eqs. taoKtoc, Tck).
__global__ void __launch_bounds__(VOX_BLOCK) k_vox_transmittance(VoxArgs A) {
    const int64_t n = (int64_t)A.n_cams * A.n_vox;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(i / A.n_vox);
        const int64_t k = i % A.n_vox;
        double x, y, z;
        voxel_centre(A, k, x, y, z);
        const HostCam& cam = A.cams[c];
        const double Dx = cam.pos[0] - x, Dy = cam.pos[1] - y, Dz = cam.pos[2] - z;
        const double len = sqrt(Dx * Dx + Dy * Dy + Dz * Dz);
        double tau = 0.0;
        if (len > 0.0)
            seg_walk(A, x, y, z, Dx / len, Dy / len, Dz / len, len,
                     [&](int64_t m, double l) { tau += A.beta[m] * l; });
        A.T[i] = exp(-tau);
    }
}

// i_c(p) = 1/(n^2 V) sum_rho sum_k l_rho(k) j_c(k) beta(k) T_c(k).
__global__ void __launch_bounds__(VOX_BLOCK) k_vox_project(VoxArgs A) {
    const double scale = 1.0 / ((double)A.n_side * A.n_side * A.dx * A.dy * A.dz);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < A.n_pix;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int c = camera_of_pixel(A, p);
        const HostCam& cam = A.cams[c];
        const int64_t lp = p - cam.pix_off;
        const int row = (int)(lp / cam.width), col = (int)(lp % cam.width);
        const double* jc = A.j + (int64_t)c * A.n_vox;
        const double* Tc = A.T + (int64_t)c * A.n_vox;
        double acc = 0.0;
        for (int b = 0; b < A.n_side; ++b)
            for (int a = 0; a < A.n_side; ++a) {
                double vx, vy, vz;
                subpixel_dir(cam, row, col, a, b, A.n_side, vx, vy, vz);
                seg_walk(A, cam.pos[0], cam.pos[1], cam.pos[2], vx, vy, vz, INFINITY,
                         [&](int64_t k, double l) { acc += l * jc[k] * A.beta[k] * Tc[k]; });
            }
        A.images[p] = acc * scale;
    }
}

// B_c = Pi_c^T dl_c: every sub-pixel ray scatters dl(p) l / (n^2 V).
__global__ void __launch_bounds__(VOX_BLOCK) k_vox_backproject(VoxArgs A) {
    const double scale = 1.0 / ((double)A.n_side * A.n_side * A.dx * A.dy * A.dz);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < A.n_pix;
         p += (int64_t)gridDim.x * blockDim.x) {
        const double g = A.dl[p] * scale;
        if (g == 0.0) continue;
        const int c = camera_of_pixel(A, p);
        const HostCam& cam = A.cams[c];
        const int64_t lp = p - cam.pix_off;
        const int row = (int)(lp / cam.width), col = (int)(lp % cam.width);
        double* Bc = A.B + (int64_t)c * A.n_vox;
        for (int b = 0; b < A.n_side; ++b)
            for (int a = 0; a < A.n_side; ++a) {
                double vx, vy, vz;
                subpixel_dir(cam, row, col, a, b, A.n_side, vx, vy, vz);
                seg_walk(A, cam.pos[0], cam.pos[1], cam.pos[2], vx, vy, vz, INFINITY,
                         [&](int64_t k, double l) { unsafeAtomicAdd(Bc + k, g * l); });
            }
    }
}

// grad(k) += T j B; then the line of sight from the centre of k to the
// camera takes -T beta j B times its length in every voxel it crosses.
__global__ void __launch_bounds__(VOX_BLOCK) k_vox_los_adjoint(VoxArgs A) {
    const int64_t n = (int64_t)A.n_cams * A.n_vox;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double bj = A.B[i] * A.j[i];
        if (bj == 0.0) continue;
        const int c = (int)(i / A.n_vox);
        const int64_t k = i % A.n_vox;
        const double T = A.T[i];
        unsafeAtomicAdd(A.grad + k, T * bj);
        const double w = T * A.beta[k] * bj;
        if (w == 0.0) continue;
        double x, y, z;
        voxel_centre(A, k, x, y, z);
        const HostCam& cam = A.cams[c];
        const double Dx = cam.pos[0] - x, Dy = cam.pos[1] - y, Dz = cam.pos[2] - z;
        const double len = sqrt(Dx * Dx + Dy * Dy + Dz * Dz);
        if (!(len > 0.0)) continue;
        seg_walk(A, x, y, z, Dx / len, Dy / len, Dz / len, len,
                 [&](int64_t m, double l) { unsafeAtomicAdd(A.grad + m, -w * l); });
    }
}

int grid_for(int64_t n) { return (int)((n + VOX_BLOCK - 1) / VOX_BLOCK < 65536 ? (n + VOX_BLOCK - 1) / VOX_BLOCK : 65536); }

}  // namespace

hipError_t launch_vox_cams(const CamChunk& chunk, HostCam* dev, hipStream_t s) {
    hipLaunchKernelGGL(k_vox_cams, dim3(1), dim3(64), 0, s, chunk, dev);
    return hipGetLastError();
}

hipError_t launch_vox_transmittance(const VoxArgs& a, hipStream_t s) {
    const int64_t n = (int64_t)a.n_cams * a.n_vox;
    if (n > 0) hipLaunchKernelGGL(k_vox_transmittance, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vox_project(const VoxArgs& a, hipStream_t s) {
    if (a.n_pix > 0) hipLaunchKernelGGL(k_vox_project, dim3(grid_for(a.n_pix)), dim3(VOX_BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vox_backproject(const VoxArgs& a, hipStream_t s) {
    if (a.n_pix > 0) hipLaunchKernelGGL(k_vox_backproject, dim3(grid_for(a.n_pix)), dim3(VOX_BLOCK), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vox_los_adjoint(const VoxArgs& a, hipStream_t s) {
    const int64_t n = (int64_t)a.n_cams * a.n_vox;
    if (n > 0) hipLaunchKernelGGL(k_vox_los_adjoint, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace mcrt
