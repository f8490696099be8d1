// C ABI of the gfx950 renderer: argument validation, stream-ordered scratch,
// camera-table upload and kernel launches.  See include/mcrt.h for the
// contract of every entry point.
#include <cmath>
#include <cstring>
#include <vector>

#include "mcrt_internal.hpp"

using namespace mcrt;

namespace {

constexpr double PI = 3.14159265358979323846;

int map_err(hipError_t e) {
    if (e == hipSuccess) return MC_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return MC_ERR_OUT_OF_MEMORY;
    if (e == hipErrorNoDevice || e == hipErrorInvalidDevice) return MC_ERR_NO_DEVICE;
    return MC_ERR_HIP;
}

#define CHECK_HIP(expr)                        \
    do {                                       \
        hipError_t e_ = (expr);                \
        if (e_ != hipSuccess) {                \
            rc = map_err(e_);                  \
            goto done;                         \
        }                                      \
    } while (0)

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int validate(const mc_grid* g, const void* beta, int n_cams, const mc_camera* cams, const mc_params* p) {
    if (!g || !beta || !cams || !p) return MC_ERR_INVALID_ARG;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return MC_ERR_INVALID_ARG;
    if ((int64_t)g->nx * g->ny * g->nz >= (int64_t)1 << 31) return MC_ERR_INVALID_ARG;
    // the local-estimate queue packs a voxel as 11 + 11 + 10 bits
    if (g->nx > 2048 || g->ny > 2048 || g->nz > 1024) return MC_ERR_INVALID_ARG;
    if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->dz)) return MC_ERR_INVALID_ARG;
    if (n_cams < 1) return MC_ERR_INVALID_ARG;
    int64_t npix = 0;
    for (int i = 0; i < n_cams; ++i) {
        const mc_camera& c = cams[i];
        if (c.width < 1 || c.height < 1) return MC_ERR_INVALID_ARG;
        if (!finite_pos(c.fx) || !finite_pos(c.fy) || !std::isfinite(c.cx) || !std::isfinite(c.cy))
            return MC_ERR_INVALID_ARG;
        for (double v : c.pos) if (!std::isfinite(v)) return MC_ERR_INVALID_ARG;
        for (double v : c.R) if (!std::isfinite(v)) return MC_ERR_INVALID_ARG;
        npix += (int64_t)c.width * c.height;
        if (npix >= (int64_t)1 << 31) return MC_ERR_INVALID_ARG;
    }
    if (!(p->albedo >= 0.0 && p->albedo <= 1.0)) return MC_ERR_INVALID_ARG;
    if (!(p->g > -1.0 && p->g < 1.0)) return MC_ERR_INVALID_ARG;
    if (!(p->sun_zenith >= 0.0 && p->sun_zenith < 0.5 * PI)) return MC_ERR_INVALID_ARG;
    if (!std::isfinite(p->sun_azimuth)) return MC_ERR_INVALID_ARG;
    if (!(p->rr_weight > 0.0 && p->rr_weight <= 1.0)) return MC_ERR_INVALID_ARG;
    if (p->max_events < 1) return MC_ERR_INVALID_ARG;
    if (p->transport != MC_FP32 && p->transport != MC_FP64) return MC_ERR_INVALID_ARG;
    if (p->tally != MC_TALLY_F64 && p->tally != MC_TALLY_KAHAN32) return MC_ERR_INVALID_ARG;
    return MC_OK;
}

int64_t pixel_count(int n_cams, const mc_camera* cams) {
    int64_t n = 0;
    for (int i = 0; i < n_cams; ++i) n += (int64_t)cams[i].width * cams[i].height;
    return n;
}

// A pointer the kernels will dereference must be device memory (or managed
// memory) of the current device.
bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

struct Scratch {
    char* base = nullptr;
    size_t off = 0;
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
        return p;
    }
};

size_t round256(size_t n) { return (n + 255) & ~(size_t)255; }

// One call of the transport kernel with all its preparation.
template <typename Real>
int run(int mode, const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
        const mc_params* prm, double* images, double* images_m2, const double* dl, double* grad, mc_stats* stats,
        uint64_t first_pid, uint32_t trace_count, uint32_t max_rec, mc_event* ev, int32_t* pix,
        mc_path* paths, hipStream_t stream) {
    int rc = MC_OK;
    const int64_t n_pix = pixel_count(n_cams, cams);
    const int64_t n_vox = (int64_t)grid->nx * grid->ny * grid->nz;
    const int tally = prm->tally == MC_TALLY_KAHAN32 ? TALLY_K32 : TALLY_F64;
    const bool k32 = tally == TALLY_K32 && mode != MODE_TRACE;

    // occupancy-mask cells: 2^sh voxels per axis, coarsened along the axis
    // with the most cells until the mask fits the kernels' LDS copy
    int sh[3] = {0, 0, 0};
    const int nn[3] = {grid->nx, grid->ny, grid->nz};
    auto ncell = [&](int a) { return (int64_t)((nn[a] + (1 << sh[a]) - 1) >> sh[a]); };
    while (ncell(0) * ncell(1) * ncell(2) > (int64_t)MASK_WORDS * 32) {
        int a = 0;
        if (ncell(1) > ncell(a)) a = 1;
        if (ncell(2) > ncell(a)) a = 2;
        ++sh[a];
    }
    const int64_t mask_words = (ncell(0) * ncell(1) * ncell(2) + 31) / 32;

    size_t bytes = round256(sizeof(unsigned long long) * (1 + ST_N)) +
                   round256(sizeof(DevCam<Real>) * n_cams) + round256(sizeof(NormCam) * n_cams) +
                   round256(sizeof(uint32_t) * mask_words);
    if (mode == MODE_GRAD) bytes += round256(sizeof(double) * n_pix);
    if (k32 && mode == MODE_RENDER) bytes += round256(sizeof(float) * 2 * n_pix);
    if (k32 && mode == MODE_GRAD) bytes += round256(sizeof(float) * 2 * n_vox);
    bytes += 256;

    Scratch S;
    KArgs<Real> A;
    std::memset(&A, 0, sizeof(A));
    unsigned long long* counters = nullptr;
    DevCam<Real>* dcams = nullptr;
    NormCam* ncams = nullptr;
    unsigned long long host_counters[1 + ST_N];
    double base_norm = 0.0;
    int dev = 0, n_cu = 0, per_cu = 0, grid_blocks = 1;
    const uint64_t n_norm = prm->n_photons_norm ? prm->n_photons_norm : prm->n_photons;

    CHECK_HIP(hipGetDevice(&dev));
    CHECK_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    CHECK_HIP(hipMallocAsync((void**)&S.base, bytes, stream));
    counters = S.take<unsigned long long>(1 + ST_N);
    dcams = S.take<DevCam<Real>>(n_cams);
    ncams = S.take<NormCam>(n_cams);

    // camera tables, passed to a writer kernel by value in chunks
    {
        int64_t off = 0;
        for (int first = 0; first < n_cams; first += CAM_CHUNK) {
            CamChunk ch;
            std::memset(&ch, 0, sizeof(ch));
            ch.first = first;
            ch.n = n_cams - first < CAM_CHUNK ? n_cams - first : CAM_CHUNK;
            ch.dx = grid->dx;
            ch.dy = grid->dy;
            ch.dz = grid->dz;
            for (int i = 0; i < ch.n; ++i) {
                const mc_camera& c = cams[first + i];
                HostCam& h = ch.c[i];
                std::memcpy(h.pos, c.pos, sizeof(h.pos));
                std::memcpy(h.R, c.R, sizeof(h.R));
                h.fx = c.fx;
                h.fy = c.fy;
                h.cx = c.cx;
                h.cy = c.cy;
                h.width = c.width;
                h.height = c.height;
                h.pix_off = off;
                off += (int64_t)c.width * c.height;
            }
            CHECK_HIP(launch_write_cams<Real>(ch, dcams, ncams, stream));
        }
    }
    CHECK_HIP(launch_fill_u64(counters, 1 + ST_N, stream));

    A.G.nx = grid->nx;
    A.G.ny = grid->ny;
    A.G.nz = grid->nz;
    A.G.nxy = grid->nx * grid->ny;
    A.G.dx = (Real)grid->dx;
    A.G.dy = (Real)grid->dy;
    A.G.dz = (Real)grid->dz;
    A.G.idx = (Real)(1.0 / grid->dx);
    A.G.idy = (Real)(1.0 / grid->dy);
    A.G.idz = (Real)(1.0 / grid->dz);
    A.beta = static_cast<const Real*>(beta);
    A.cams = dcams;
    A.n_cams = n_cams;
    A.wsx = (Real)(-std::sin(prm->sun_zenith) * std::cos(prm->sun_azimuth));
    A.wsy = (Real)(-std::sin(prm->sun_zenith) * std::sin(prm->sun_azimuth));
    A.wsz = (Real)(-std::cos(prm->sun_zenith));
    A.albedo = (Real)prm->albedo;
    A.g = (Real)prm->g;
    A.rr = (Real)prm->rr_weight;
    A.max_events = prm->max_events;
    A.seed = prm->seed;
    A.pid0 = prm->photon_offset;
    A.n_photons = prm->n_photons;
    A.work = counters;
    A.stats = counters + 1;
    A.n_pix = n_pix;
    A.n_vox = n_vox;
    A.mshx = sh[0];
    A.mshy = sh[1];
    A.mshz = sh[2];
    A.mncx = (int)ncell(0);
    A.mncy = (int)ncell(1);
    A.mask_words = (int)mask_words;
    A.mask_fine = (sh[0] | sh[1] | sh[2]) == 0;
    A.grad_lds = mode == MODE_GRAD &&
                 ((mask_words + 1) & ~(int64_t)1) * 4 + n_vox * (int64_t)sizeof(double) <= GRAD_LDS_BYTES;
    CHECK_HIP(transport_occupancy<Real>(A, mode, tally, &per_cu));
    if (mode != MODE_TRACE) {
        uint32_t* mask = S.take<uint32_t>(mask_words);
        A.mask = mask;
        CHECK_HIP(launch_build_mask<Real>(A, mask, (int)ncell(2), stream));
    }
    base_norm = n_norm ? std::cos(prm->sun_zenith) * (grid->nx * grid->dx) * (grid->ny * grid->dy) / (double)n_norm
                       : 0.0;

    if (mode == MODE_RENDER) {
        A.img = images;
        A.img_m2 = images_m2;
        if (images_m2) CHECK_HIP(launch_fill_f64(images_m2, n_pix, stream));
        if (k32) {
            A.img32 = S.take<float>(2 * n_pix);
            CHECK_HIP(launch_fill_f32(A.img32, 2 * n_pix, stream));
        } else {
            CHECK_HIP(launch_fill_f64(images, n_pix, stream));
        }
    } else if (mode == MODE_GRAD) {
        double* gw = S.take<double>(n_pix);
        CHECK_HIP(launch_grad_weights(gw, dl, ncams, n_cams, n_pix, base_norm, stream));
        A.gw = gw;
        A.grad = grad;
        if (k32) {
            A.grad32 = S.take<float>(2 * n_vox);
            CHECK_HIP(launch_fill_f32(A.grad32, 2 * n_vox, stream));
        } else {
            CHECK_HIP(launch_fill_f64(grad, n_vox, stream));
        }
    } else {
        A.first_pid = first_pid;
        A.trace_count = trace_count;
        A.max_rec = max_rec;
        A.ev = ev;
        A.pix = pix;
        A.paths = paths;
    }

    if (mode == MODE_TRACE) {
        grid_blocks = (int)((trace_count + BLOCK - 1) / BLOCK);
    } else {
        const int64_t full = (int64_t)n_cu * (per_cu > 0 ? per_cu : 1);
        const int64_t need = (int64_t)((prm->n_photons + BLOCK - 1) / BLOCK);
        grid_blocks = (int)(need < full ? need : full);
    }
    if (grid_blocks > 0 && (mode == MODE_TRACE || prm->n_photons > 0))
        CHECK_HIP(launch_transport<Real>(A, mode, tally, grid_blocks, stream));

    if (mode == MODE_RENDER) {
        if (k32) CHECK_HIP(launch_kahan_reduce(images, A.img32, n_pix, stream));
        CHECK_HIP(launch_normalize(images, ncams, n_cams, n_pix, base_norm, 1, stream));
        if (images_m2) CHECK_HIP(launch_normalize(images_m2, ncams, n_cams, n_pix, base_norm, 2, stream));
    } else if (mode == MODE_GRAD && k32) {
        CHECK_HIP(launch_kahan_reduce(grad, A.grad32, n_vox, stream));
    }

    if (stats || mode == MODE_TRACE) {
        CHECK_HIP(hipMemcpyAsync(host_counters, counters, sizeof(host_counters), hipMemcpyDeviceToHost, stream));
        CHECK_HIP(hipStreamSynchronize(stream));
        if (stats) {
            stats->photons = mode == MODE_TRACE ? trace_count : prm->n_photons;
            stats->events = host_counters[1 + ST_EVENTS];
            stats->le_jobs = host_counters[1 + ST_LE];
            stats->vox_free = host_counters[1 + ST_VFREE];
            stats->vox_conn = host_counters[1 + ST_VCONN];
            stats->esc_top = host_counters[1 + ST_TOP];
            stats->esc_bottom = host_counters[1 + ST_BOTTOM];
            stats->esc_side = host_counters[1 + ST_SIDE];
            stats->rr_killed = host_counters[1 + ST_RR];
            stats->capped = host_counters[1 + ST_CAP];
        }
    }

done:
    if (S.base) {
        hipError_t e = hipFreeAsync(S.base, stream);
        if (rc == MC_OK && e != hipSuccess) rc = map_err(e);
    }
    return rc;
}

int precheck_device() {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n < 1) {
        (void)hipGetLastError();
        return MC_ERR_NO_DEVICE;
    }
    return MC_OK;
}

}  // namespace

extern "C" {

int mc_device_count(void) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

const char* mc_error_string(int code) {
    switch (code) {
        case MC_OK: return "success";
        case MC_ERR_INVALID_ARG: return "invalid argument";
        case MC_ERR_NO_DEVICE: return "no HIP device";
        case MC_ERR_HIP: return "HIP runtime error";
        case MC_ERR_OUT_OF_MEMORY: return "out of device memory";
        default: return "unknown status code";
    }
}

int mc_render(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams, const mc_params* params,
              double* images, mc_stats* stats, void* hip_stream) {
    return mc_render_moments(grid, beta, n_cams, cams, params, images, nullptr, stats, hip_stream);
}

int mc_render_moments(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
                      const mc_params* params, double* images, double* images_m2, mc_stats* stats,
                      void* hip_stream) {
    int rc = validate(grid, beta, n_cams, cams, params);
    if (rc != MC_OK) return rc;
    if (!images) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(images)) return MC_ERR_INVALID_ARG;
    if (images_m2 && !is_device_ptr(images_m2)) return MC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (params->transport == MC_FP64)
        return run<double>(MODE_RENDER, grid, beta, n_cams, cams, params, images, images_m2, nullptr, nullptr, stats,
                           0, 0, 0, nullptr, nullptr, nullptr, s);
    return run<float>(MODE_RENDER, grid, beta, n_cams, cams, params, images, images_m2, nullptr, nullptr, stats, 0,
                      0, 0, nullptr, nullptr, nullptr, s);
}

int mc_grad_beta(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams, const mc_params* params,
                 const double* dl_dimages, double* grad_beta, mc_stats* stats, void* hip_stream) {
    int rc = validate(grid, beta, n_cams, cams, params);
    if (rc != MC_OK) return rc;
    if (!dl_dimages || !grad_beta) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(dl_dimages) || !is_device_ptr(grad_beta)) return MC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (params->transport == MC_FP64)
        return run<double>(MODE_GRAD, grid, beta, n_cams, cams, params, nullptr, nullptr, dl_dimages, grad_beta,
                           stats, 0, 0, 0, nullptr, nullptr, nullptr, s);
    return run<float>(MODE_GRAD, grid, beta, n_cams, cams, params, nullptr, nullptr, dl_dimages, grad_beta, stats,
                      0, 0, 0, nullptr, nullptr, nullptr, s);
}

int mc_trace_paths(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams, const mc_params* params,
                   uint64_t first_pid, uint32_t count, uint32_t max_rec, mc_event* events, int32_t* pix,
                   mc_path* paths, void* hip_stream) {
    int rc = validate(grid, beta, n_cams, cams, params);
    if (rc != MC_OK) return rc;
    if (count > 0 && !paths) return MC_ERR_INVALID_ARG;
    if (count > 0 && max_rec > 0 && !events) return MC_ERR_INVALID_ARG;
    if (count > (1u << 30) || (uint64_t)count * max_rec >= ((uint64_t)1 << 40)) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta)) return MC_ERR_INVALID_ARG;
    if (count > 0 && !is_device_ptr(paths)) return MC_ERR_INVALID_ARG;
    if (events && !is_device_ptr(events)) return MC_ERR_INVALID_ARG;
    if (pix && !is_device_ptr(pix)) return MC_ERR_INVALID_ARG;
    if (count == 0) return MC_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (params->transport == MC_FP64)
        return run<double>(MODE_TRACE, grid, beta, n_cams, cams, params, nullptr, nullptr, nullptr, nullptr,
                           nullptr, first_pid, count, max_rec, events, pix, paths, s);
    return run<float>(MODE_TRACE, grid, beta, n_cams, cams, params, nullptr, nullptr, nullptr, nullptr, nullptr,
                      first_pid, count, max_rec, events, pix, paths, s);
}

}  // extern "C"
