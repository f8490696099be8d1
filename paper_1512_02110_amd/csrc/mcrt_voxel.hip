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
        const double* qc = A.q ? A.q + (int64_t)c * A.n_vox : nullptr;
        unsafeAtomicAdd(A.grad + k, (qc ? qc[k] : 1.0) * T * bj);
        const double w = T * A.beta[k] * bj;
        if (w == 0.0) continue;
        double x, y, z;
        voxel_centre(A, k, x, y, z);
        const HostCam& cam = A.cams[c];
        const double Dx = cam.pos[0] - x, Dy = cam.pos[1] - y, Dz = cam.pos[2] - z;
        const double len = sqrt(Dx * Dx + Dy * Dy + Dz * Dz);
        if (!(len > 0.0)) continue;
        seg_walk(A, x, y, z, Dx / len, Dy / len, Dz / len, len,
                 [&](int64_t m, double l) { unsafeAtomicAdd(A.grad + m, -(qc ? qc[m] : 1.0) * w * l); });
    }
}

// Sec. 6: counts[c][k] += 1 for every sub-pixel ray of camera c whose length
// in voxel k exceeds 1e-9 of the shortest voxel edge (a ray that only grazes
// an edge or a corner is not counted, whatever the rounding).
__global__ void __launch_bounds__(VOX_BLOCK) k_vox_ray_counts(VoxArgs A, double* counts) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < A.n_pix;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int c = camera_of_pixel(A, p);
        const HostCam& cam = A.cams[c];
        const int64_t lp = p - cam.pix_off;
        const int row = (int)(lp / cam.width), col = (int)(lp % cam.width);
        double* Cc = counts + (int64_t)c * A.n_vox;
        const double eps = 1e-9 * fmin(A.dx, fmin(A.dy, A.dz));
        for (int b = 0; b < A.n_side; ++b)
            for (int a = 0; a < A.n_side; ++a) {
                double vx, vy, vz;
                subpixel_dir(cam, row, col, a, b, A.n_side, vx, vy, vz);
                seg_walk(A, cam.pos[0], cam.pos[1], cam.pos[2], vx, vy, vz, INFINITY, [&](int64_t k, double l) {
                    if (l > eps) unsafeAtomicAdd(Cc + k, 1.0);
                });
            }
    }
}

// q = 1 / count where a ray passes, else 0 (in place).
__global__ void k_vox_invert(double* x, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = x[i] > 0.0 ? 1.0 / x[i] : 0.0;
}

// Block sum of v into *out (one device atomic per block).
__device__ void block_sum_add(double v, double* s_red, double* out) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_red[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += s_red[w];
        unsafeAtomicAdd(out, t);
    }
}

// 7-point Laplacian in voxel units at (ix, iy, iz); a neighbour outside the
// domain takes the centre's value (no flux through the boundary).
__device__ double lap_at(const double* f, int nx, int ny, int nz, int ix, int iy, int iz) {
    const int64_t nxy = (int64_t)nx * ny;
    const int64_t k = ix + (int64_t)nx * iy + nxy * iz;
    const double c = f[k];
    double s = -6.0 * c;
    s += ix > 0 ? f[k - 1] : c;
    s += ix < nx - 1 ? f[k + 1] : c;
    s += iy > 0 ? f[k - nx] : c;
    s += iy < ny - 1 ? f[k + nx] : c;
    s += iz > 0 ? f[k - nxy] : c;
    s += iz < nz - 1 ? f[k + nxy] : c;
    return s;
}

// Sec. 6, Psi = |W Lap beta|^2: r = W^2 Lap beta (scratch), *value += Psi.
__global__ void __launch_bounds__(VOX_BLOCK) k_reg_residual(int nx, int ny, int nz, const double* beta,
                                                            const double* w_layer, double* r, double* value) {
    __shared__ double s_red[VOX_BLOCK / 64];
    const int64_t n = (int64_t)nx * ny * nz, nxy = (int64_t)nx * ny;
    double acc = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int ix = (int)(k % nx), iy = (int)((k / nx) % ny), iz = (int)(k / nxy);
        const double w = w_layer ? w_layer[iz] : 1.0;
        const double l = lap_at(beta, nx, ny, nz, ix, iy, iz);
        acc += (w * l) * (w * l);
        r[k] = w * w * l;
    }
    if (value) block_sum_add(acc, s_red, value);
}

// grad += eta * 2 Lap r (Lap is symmetric).
__global__ void __launch_bounds__(VOX_BLOCK) k_reg_grad(int nx, int ny, int nz, const double* r, double eta,
                                                        double* grad) {
    const int64_t n = (int64_t)nx * ny * nz, nxy = (int64_t)nx * ny;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int ix = (int)(k % nx), iy = (int)((k / nx) % ny), iz = (int)(k / nxy);
        grad[k] += eta * 2.0 * lap_at(r, nx, ny, nz, ix, iy, iz);
    }
}

// Eq. (Cost) data term: r = M (i - measured); dl = 2 M r; *loss += sum r^2.
__global__ void __launch_bounds__(VOX_BLOCK) k_image_residual(int64_t n, const double* img, const double* meas,
                                                              const double* mask, double* dl, double* loss) {
    __shared__ double s_red[VOX_BLOCK / 64];
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const double m = mask ? mask[p] : 1.0;
        const double r = m * (img[p] - meas[p]);
        acc += r * r;
        dl[p] = 2.0 * m * r;
    }
    if (loss) block_sum_add(acc, s_red, loss);
}

// Eq. (GD) projected on the non-negative set: beta = max(beta - delta g, 0).
__global__ void k_gd_step(int64_t n, double* beta, const double* g, double delta) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const double b = beta[k] - delta * g[k];
        beta[k] = b > 0.0 ? b : 0.0;
    }
}

// Largest masked pixel (values are >= 0: the bit pattern orders like the
// value, so an integer max does).
__global__ void __launch_bounds__(VOX_BLOCK) k_masked_max(int64_t n, const double* img, const double* mask,
                                                          unsigned long long* mx) {
    unsigned long long best = 0ull;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const double v = (mask ? mask[p] : 1.0) * img[p];
        if (v > 0.0) {
            const unsigned long long u = (unsigned long long)__double_as_longlong(v);
            best = u > best ? u : best;
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long t = __shfl_down(best, o);
        best = t > best ? t : best;
    }
    if ((threadIdx.x & 63) == 0 && best) atomicMax(mx, best);
}

// Eq. (noise) with the caller's N(0,1) draws.
__global__ void k_camera_noise(int64_t n, const double* img, const double* normals,
                               const unsigned long long* mx, double* out, double* scale_out) {
    const double m = __longlong_as_double((long long)*mx);
    const double scale = m > 0.0 ? 1024.0 / m : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0 && scale_out) *scale_out = scale;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const double x = floor(img[p] * scale + 0.4 * normals[p] + 0.5);
        out[p] = x < 0.0 ? 0.0 : (x > 1024.0 ? 1024.0 : x);
    }
}

// Sec. 7: sums |b|, |t|, |b - t| into acc[0..2].
__global__ void __launch_bounds__(VOX_BLOCK) k_recovery_sums(int64_t n, const double* b, const double* t,
                                                             double* acc) {
    __shared__ double s_red[VOX_BLOCK / 64];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        a0 += fabs(b[k]);
        a1 += fabs(t[k]);
        a2 += fabs(b[k] - t[k]);
    }
    block_sum_add(a0, s_red, acc);
    __syncthreads();
    block_sum_add(a1, s_red, acc + 1);
    __syncthreads();
    block_sum_add(a2, s_red, acc + 2);
}

__global__ void k_d2f(int64_t n, const double* in, float* out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)in[i];
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

hipError_t launch_vox_ray_counts(const VoxArgs& a, double* counts, hipStream_t s) {
    if (a.n_pix > 0) hipLaunchKernelGGL(k_vox_ray_counts, dim3(grid_for(a.n_pix)), dim3(VOX_BLOCK), 0, s, a, counts);
    return hipGetLastError();
}

hipError_t launch_vox_invert(double* x, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_vox_invert, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, x, n);
    return hipGetLastError();
}

hipError_t launch_reg(int nx, int ny, int nz, const double* beta, const double* w_layer, double eta, double* r,
                      double* grad, double* value, hipStream_t s) {
    const int64_t n = (int64_t)nx * ny * nz;
    hipLaunchKernelGGL(k_reg_residual, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, nx, ny, nz, beta, w_layer, r, value);
    if (grad) hipLaunchKernelGGL(k_reg_grad, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, nx, ny, nz, r, eta, grad);
    return hipGetLastError();
}

hipError_t launch_image_residual(int64_t n, const double* img, const double* meas, const double* mask, double* dl,
                                 double* loss, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_image_residual, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, n, img, meas, mask, dl, loss);
    return hipGetLastError();
}

hipError_t launch_gd_step(int64_t n, double* beta, const double* g, double delta, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_gd_step, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, n, beta, g, delta);
    return hipGetLastError();
}

hipError_t launch_camera_noise(int64_t n, const double* img, const double* mask, const double* normals,
                               unsigned long long* mx, double* out, double* scale_out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_masked_max, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, n, img, mask, mx);
    hipLaunchKernelGGL(k_camera_noise, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, n, img, normals, mx, out, scale_out);
    return hipGetLastError();
}

hipError_t launch_d2f(int64_t n, const double* in, float* out, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_d2f, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, n, in, out);
    return hipGetLastError();
}

hipError_t launch_recovery_sums(int64_t n, const double* b, const double* t, double* acc, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_recovery_sums, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, n, b, t, acc);
    return hipGetLastError();
}

hipError_t launch_vox_los_adjoint(const VoxArgs& a, hipStream_t s) {
    const int64_t n = (int64_t)a.n_cams * a.n_vox;
    if (n > 0) hipLaunchKernelGGL(k_vox_los_adjoint, dim3(grid_for(n)), dim3(VOX_BLOCK), 0, s, a);
    return hipGetLastError();
}

}  // namespace mcrt
