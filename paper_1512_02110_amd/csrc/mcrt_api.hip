// C ABI of the gfx950 renderer: argument validation, stream-ordered scratch,
// camera-table upload and kernel launches.  See include/mcrt.h for the
// contract of every entry point.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "mcrt_internal.hpp"

using namespace mcrt;

// The rays of a render kept for a later gradient (mc_render_tape): one
// slice of rw records per wavefront of the render, and what the render was
// called with, so that mc_grad_beta_tape can check that it asks for the
// gradient of the same render.
struct mc_tape {
    uint32_t magic;
    int device;
    mc_grid grid;
    mc_params params;
    int n_cams;
    uint64_t cam_hash;          // FNV-1a of the camera structs
    size_t rec_bytes;           // bytes of one record (precision)
    void* rec;                  // device: nw slices of rw records
    uint32_t* wave_count;       // device: [nw] records per slice, then the overflow flag
    int nw;
    uint32_t rw;
    unsigned long long counters[1 + ST_N];  // the render's counters (host copy)
};

// Device scratch of mc_render_noalloc, for callers that cannot allocate: a
// file-scope array of NOALLOC_SCRATCH_BYTES, one copy per device, held until
// the process ends.  In host code its name is only a host-side stand-in:
// every kernel argument or copy uses the device address that
// hipGetSymbolAddress returned for the current device (g_noalloc_ptr).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

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

int validate_scene(const mc_grid* g, const void* beta, int n_cams, const mc_camera* cams) {
    if (!g || !beta || !cams) return MC_ERR_INVALID_ARG;
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return MC_ERR_INVALID_ARG;
    if ((int64_t)g->nx * g->ny * g->nz >= (int64_t)1 << 31) return MC_ERR_INVALID_ARG;
    // the local-estimate queue packs a voxel as 11 + 11 + 10 bits
    if (g->nx > 2048 || g->ny > 2048 || g->nz > 1024) return MC_ERR_INVALID_ARG;
    if (!finite_pos(g->dx) || !finite_pos(g->dy) || !finite_pos(g->dz)) return MC_ERR_INVALID_ARG;
    // camera indices travel as 16-bit values through the job queue
    if (n_cams < 1 || n_cams > 65535) return MC_ERR_INVALID_ARG;
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
    return MC_OK;
}

int validate(const mc_grid* g, const void* beta, int n_cams, const mc_camera* cams, const mc_params* p) {
    int rc = validate_scene(g, beta, n_cams, cams);
    if (rc != MC_OK) return rc;
    if (!p) return MC_ERR_INVALID_ARG;
    if (!(p->albedo >= 0.0 && p->albedo <= 1.0)) return MC_ERR_INVALID_ARG;
    if (!(p->g > -1.0 && p->g < 1.0)) return MC_ERR_INVALID_ARG;
    if (!(p->sun_zenith >= 0.0 && p->sun_zenith < 0.5 * PI)) return MC_ERR_INVALID_ARG;
    if (!std::isfinite(p->sun_azimuth)) return MC_ERR_INVALID_ARG;
    if (!(p->rr_weight > 0.0 && p->rr_weight <= 1.0)) return MC_ERR_INVALID_ARG;
    if (p->max_events < 1) return MC_ERR_INVALID_ARG;
    if (p->transport != MC_FP32 && p->transport != MC_FP64 && p->transport != MC_MIXED) return MC_ERR_INVALID_ARG;
    if (p->tally != MC_TALLY_F64 && p->tally != MC_TALLY_KAHAN32) return MC_ERR_INVALID_ARG;
    if (p->tape_limit < 0) return MC_ERR_INVALID_ARG;
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

// MC_PLAIN_WALK_LOADS=1: connection walks use plain loads whatever the grid's
// size (the path of grids too large for a buffer, testable on small ones)
bool plain_walk_loads() {
    const char* v = std::getenv("MC_PLAIN_WALK_LOADS");
    return v && v[0] == '1';
}

// An air + aerosol mixture: device fields of the reference channel and the
// channel's aerosol cross-section ratio (Eq. channelBeta).
// The gather capture (mc_capture_gathers): where the walks' loaded indices go.
struct CaptureArgs {
    uint32_t* idx;
    uint32_t* steps;
    uint32_t first, n_steps, max_waves;
    uint32_t n_waves;  // out: wavefronts of the launch
};

struct MixIn {
    const double* air;
    const double* aer;
    double sig;
    int full;  // gradient: 1 full (path scores), 0 surrogate
};

// Device memory of the library comes from one memory pool per device that
// keeps what the calls free (release threshold: unlimited), so that the
// tapes and bins, tens of GB each, are not mapped and unmapped on every
// call; mc_release_memory hands the cached memory back to the device.  The
// same lock guards the tape sizing hint (rays per photon of the busiest
// wavefront of the last kept render on the device, and the key of the
// workload it was measured on: grid, cameras, albedo, phase and sun).
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
hipMemPool_t g_pool[MAX_DEVICES] = {};
double g_tape_rate[MAX_DEVICES] = {};
uint64_t g_tape_key[MAX_DEVICES] = {};
void* g_noalloc_ptr[MAX_DEVICES] = {};  // device address of `scratch` on each device

// Device address of the no-allocation scratch on the current device, looked
// up once per device (with that device current).
hipError_t noalloc_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_noalloc_ptr[dev] = p;
    }
    *out = g_noalloc_ptr[dev];
    return hipSuccess;
}

hipError_t lib_pool(int dev, hipMemPool_t* out) {
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_pool[dev]) {
        hipMemPoolProps props;
        std::memset(&props, 0, sizeof(props));
        props.allocType = hipMemAllocationTypePinned;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = dev;
        hipMemPool_t p = nullptr;
        hipError_t e = hipMemPoolCreate(&p, &props);
        if (e != hipSuccess) return e;
        uint64_t keep_all = ~0ull;
        e = hipMemPoolSetAttribute(p, hipMemPoolAttrReleaseThreshold, &keep_all);
        if (e != hipSuccess) {
            (void)hipMemPoolDestroy(p);
            return e;
        }
        g_pool[dev] = p;
    }
    *out = g_pool[dev];
    return hipSuccess;
}

// Stream-ordered allocation from the library's pool of the current device
// (released with hipFreeAsync).
hipError_t lib_alloc(void** ptr, size_t bytes, hipStream_t stream) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipMemPool_t pool = nullptr;
    if ((e = lib_pool(dev, &pool)) != hipSuccess) return e;
    return hipMallocFromPoolAsync(ptr, bytes, pool, stream);
}

// The two large buffers of the library, kept per device between calls: the
// rays of a kept render (BUF_TAPE) and the bins (or replay tape) of a
// gradient (BUF_BINS).  Freeing and mapping buffers of tens of GB on every
// call costs hundreds of ms, so a released buffer stays cached, and a later
// request of at most its size takes it back (its stream first waits for the
// work of the releasing stream).  A request while the buffer is taken (two
// tapes alive) is served from the pool.
enum { BUF_TAPE = 0, BUF_BINS = 1, N_BUFS = 2 };
struct CachedBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    bool in_use = false;
    hipEvent_t ready = nullptr;  // recorded where the last user released it
};
CachedBuf g_buf[MAX_DEVICES][N_BUFS];

hipError_t buf_acquire(int slot, size_t bytes, hipStream_t stream, void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        CachedBuf& b = g_buf[dev][slot];
        if (!b.in_use) {
            if (b.bytes < bytes) {
                if (b.ptr) {
                    (void)hipFree(b.ptr);  // waits for the device
                    b.ptr = nullptr;
                    b.bytes = 0;
                }
                if ((e = hipMalloc(&b.ptr, bytes)) != hipSuccess) {
                    b.ptr = nullptr;
                    return e;
                }
                b.bytes = bytes;
            }
            if (!b.ready) {
                if ((e = hipEventCreateWithFlags(&b.ready, hipEventDisableTiming)) != hipSuccess) return e;
            } else if ((e = hipStreamWaitEvent(stream, b.ready, 0)) != hipSuccess) {
                return e;
            }
            b.in_use = true;
            *ptr = b.ptr;
            return hipSuccess;
        }
    }
    return lib_alloc(ptr, bytes, stream);
}

void buf_release(int dev, int slot, void* ptr, hipStream_t stream) {
    if (!ptr) return;
    if (dev >= 0 && dev < MAX_DEVICES) {
        std::lock_guard<std::mutex> lock(g_mu);
        CachedBuf& b = g_buf[dev][slot];
        if (b.in_use && b.ptr == ptr) {
            (void)hipEventRecord(b.ready, stream);
            b.in_use = false;
            return;
        }
    }
    (void)hipFreeAsync(ptr, stream);
}

// Device memory a call can use: free memory plus what the library's pool
// and buffers hold unused.
hipError_t available_bytes(size_t* avail) {
    size_t free_b = 0, total_b = 0;
    hipError_t e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) return e;
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    hipMemPool_t pool = nullptr;
    if ((e = lib_pool(dev, &pool)) != hipSuccess) return e;
    uint64_t reserved = 0, used = 0;
    if (hipMemPoolGetAttribute(pool, hipMemPoolAttrReservedMemCurrent, &reserved) != hipSuccess ||
        hipMemPoolGetAttribute(pool, hipMemPoolAttrUsedMemCurrent, &used) != hipSuccess) {
        (void)hipGetLastError();
        reserved = used = 0;
    }
    *avail = free_b + (reserved > used ? (size_t)(reserved - used) : 0);
    std::lock_guard<std::mutex> lock(g_mu);
    for (int i = 0; i < N_BUFS; ++i)
        if (dev < MAX_DEVICES && !g_buf[dev][i].in_use) *avail += g_buf[dev][i].bytes;
    return hipSuccess;
}

// Tile edges of the gradient tape, as powers of two (so that the tile of a
// voxel is a shift away): columns of at most 64 voxels in z and TILE_VOX
// voxels in all.  Connection rays to cameras below or above the cloud are
// closer to vertical than to horizontal, so tall tiles are crossed by fewer
// rays more than once.
int ceil_log2(int n) {
    int s = 0;
    while ((1 << s) < n) ++s;
    return s;
}

void tape_tiles(const mc_grid* g, int& shx, int& shy, int& shz) {
    const int total = ceil_log2(TILE_VOX);
    shz = std::min(6, ceil_log2(g->nz));
    const int rest = total - shz;
    shx = std::min(ceil_log2(g->nx), (rest + 1) / 2);
    shy = std::min(ceil_log2(g->ny), rest - shx);
    if (shy < rest - shx) shx = std::min(ceil_log2(g->nx), rest - shy);
    // the deposit's padded LDS copy of a tile must fit (flat tiles of a thin
    // grid have the most padding)
    while (((1 << shx) + 1) * ((1 << shy) + 1) * (1 << shz) > TILE_LDS) {
        if (shx >= shy && shx > 0)
            --shx;
        else if (shy > 0)
            --shy;
        else
            --shz;
    }
}

constexpr int TAPE_FALLBACK = 1;

// Ray buffers of the overlapped gradient replay (each with a library stream).
// Three were 1-6% slower than two on the 64^3, 128^3 and 256x256x128
// workloads: a third replay in flight competes with the other two for the
// compute units and makes every chunk smaller (more chunks, more tails).
constexpr int REPLAY_BUFFERS = 2;
// Chunks of the replay at least: its first replay and its last chunk's
// deposits overlap nothing, so a call of a few large chunks overlaps less
// (on the 64^3 workload 4 chunks were 1.5% slower than 5).
constexpr int MIN_REPLAY_CHUNKS = 5;

// Binning blocks per wavefront slice for a pass over ns slices (at least
// BIN_BLOCKS_PER_CU blocks per CU where the slices allow), and the most
// blocks a pass can have with nw slices at most (the slice matrix's columns).
int bin_split(int ns, int n_cu) {
    const int target = BIN_BLOCKS_PER_CU * n_cu;
    return ns >= target ? 1 : std::min(BIN_SPLIT_MAX, (target + ns - 1) / ns);
}

size_t bin_blocks_max(int nw, int n_cu) { return (size_t)std::max(nw, 2 * BIN_BLOCKS_PER_CU * n_cu); }

// Bins and deposits the rays of the binning pass set up in A.tp (slices,
// records, tile counts h_count from its count pass): groups of tiles whose
// bins fit together in b_cap slots, each turned into bin slots (k_bin_scan),
// filled (k_bin, scatter pass) and deposited tile by tile (k_deposit).
template <typename Real>
int deposit_groups(KArgs<Real>& A, int tally, const std::vector<uint32_t>& h_count, uint64_t b_cap, int n_cu,
                   DepositItem* ditems, int max_items, std::vector<uint32_t>& h_bins,
                   std::vector<DepositItem>& h_items, hipStream_t stream) {
    int rc = MC_OK;
    const int nt = A.tp.n_tiles;
    for (int g0 = 0; g0 < nt;) {
        // the next group of tiles whose bins fit together
        uint64_t sum = 0;
        int g1 = g0;
        while (g1 < nt && g1 - g0 < BIN_GROUP_TILES && sum + h_count[g1] <= b_cap) sum += h_count[g1++];
        if (g1 == g0) return MC_ERR_OUT_OF_MEMORY;  // one bin larger than the space (checked by the callers)
        uint32_t o = 0;
        for (int i = g0; i < g1; ++i) {
            h_bins[i] = o;
            h_bins[nt + i] = o + h_count[i];
            o += h_count[i];
        }
        const uint64_t per = (uint64_t)DEP_ITEMS_PER_CU * n_cu;
        const uint64_t R = std::max<uint64_t>(8192, (sum + per - 1) / per);
        h_items.clear();
        for (int i = g0; i < g1; ++i)
            for (uint64_t lo = 0; lo < h_count[i]; lo += R) {
                DepositItem d;
                d.tile = i;
                d.lo = h_bins[i] + (uint32_t)lo;
                d.hi = h_bins[i] + (uint32_t)std::min<uint64_t>(h_count[i], lo + R);
                d.pad_ = 0;
                h_items.push_back(d);
            }
        // blocks start in launch order as CUs free up: the largest items
        // first, so that the last ones to start are the short remainders
        std::stable_sort(h_items.begin(), h_items.end(), [](const DepositItem& x, const DepositItem& y) {
            return x.hi - x.lo > y.hi - y.lo;
        });
        if ((int)h_items.size() > max_items) return MC_ERR_HIP;
        A.tp.t_lo = g0;
        A.tp.t_hi = g1;
        CHECK_HIP(hipMemcpyAsync(const_cast<uint32_t*>(A.tp.bin_start) + g0, h_bins.data() + g0,
                                 sizeof(uint32_t) * (g1 - g0), hipMemcpyHostToDevice, stream));
        CHECK_HIP(hipMemcpyAsync(const_cast<uint32_t*>(A.tp.tile_end) + g0, h_bins.data() + nt + g0,
                                 sizeof(uint32_t) * (g1 - g0), hipMemcpyHostToDevice, stream));
        CHECK_HIP(launch_bin_scan<Real>(A, stream));
        CHECK_HIP(launch_bin<Real>(A, true, stream));
        if (!h_items.empty()) {
            CHECK_HIP(hipMemcpyAsync(ditems, h_items.data(), sizeof(DepositItem) * h_items.size(),
                                     hipMemcpyHostToDevice, stream));
            CHECK_HIP(launch_deposit<Real>(A, tally, ditems, (int)h_items.size(), stream));
        }
        g0 = g1;
        if (g0 < nt) CHECK_HIP(hipStreamSynchronize(stream));  // host arrays are reused
    }
done:
    return rc;
}

// Gradient of a large grid through the tape, in chunks of photons:
//   1. replay the chunk (k_render, MODE_TAPE): every wavefront writes the
//      connection rays with a non-zero weight to its slice of the ray tape;
//   2. count the rays crossing each tile, per block of the binning passes
//      (k_bin, count pass), and read the totals back;
//   3. for groups of tiles whose bins fit the bin space: turn the block
//      counts into bin slots (k_bin_scan), copy the rays into the bins (k_bin,
//      scatter pass) and deposit every tile (k_deposit).
// The tape space is split between rays and bins per chunk, from the rays
// per photon of the busiest wavefront and the tile crossings per photon of
// the chunks so far, so that a chunk's bins usually fit in one group.  A
// chunk whose rays overflowed a wavefront slice, or with a tile bin larger
// than the bin space, is replayed smaller before anything of it reaches the
// gradient.  Stats of the completed chunks are summed into host_sum.
//
// With mp (full gradient of a mixture), the replay also sums every
// collision's a = gw C into the photon's row of mp->rows (chunks of at most
// mp->max_chunk photons), and each chunk that reaches the gradient is
// followed by the path scores of its photons (k_mix_path).
struct MixPath {
    double* rows;        // (cap + 1) sums per photon of the chunk
    uint32_t cap;        // collisions with a row entry of their own
    uint64_t max_chunk;  // photons the rows hold
    int grid;            // blocks of k_mix_path
};

// The rays per photon of the busiest wavefront last measured on this device
// for workload key `key` (a kept render or a replay), 0 if none.
double tape_hint(uint64_t key) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return 0.0;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_tape_key[dev] == key ? g_tape_rate[dev] : 0.0;
}

void set_tape_hint(uint64_t key, double rate) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES || !(rate > 0.0)) return;
    std::lock_guard<std::mutex> lock(g_mu);
    g_tape_rate[dev] = rate;
    g_tape_key[dev] = key;
}

// Two library streams per device for the overlapped replay (created once,
// default priority, kept until the process ends).
hipStream_t g_rstream[MAX_DEVICES][REPLAY_BUFFERS] = {};

bool replay_streams(hipStream_t out[REPLAY_BUFFERS]) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return false;
    std::lock_guard<std::mutex> lock(g_mu);
    for (int i = 0; i < REPLAY_BUFFERS; ++i) {
        if (!g_rstream[dev][i] && hipStreamCreateWithFlags(&g_rstream[dev][i], hipStreamNonBlocking) != hipSuccess) {
            (void)hipGetLastError();
            g_rstream[dev][i] = nullptr;
            return false;
        }
        out[i] = g_rstream[dev][i];
    }
    return true;
}

// The gradient replay of run_tape with REPLAY_BUFFERS ray buffers, so that
// the replay of a chunk (each buffer on a library stream of its own)
// overlaps the binning and deposits of an earlier one (on the caller's
// stream) and, above all, the tail of the previous replay: every replay
// launch ends with a few wavefronts on the last, longest photons, and the
// next launch's wavefronts fill the compute units they leave.  The tape
// space holds the ray regions of r_cap slots and the bins (b_cap slots);
// the split is fixed for the call (from the workload's measured rays per
// photon when there is one), the chunk sizes adapt to what each counted
// chunk measured.  A chunk whose rays overflowed
// a slice, or with a bin larger than the bin space, goes back to the queue
// of ranges and is replayed in halves; photon ranges may complete out of
// order (the gradient is a sum).
template <typename Real>
int run_tape_overlap(KArgs<Real> A, int tally, uint64_t n_photons, uint64_t pid0, int64_t tape_limit,
                     int max_blocks, int n_cu, unsigned long long* counters, unsigned long long* host_sum,
                     double* t_transport, double* t_tape, hipStream_t stream, uint64_t wkey,
                     const hipStream_t rs[REPLAY_BUFFERS]) {
    int rc = MC_OK;
    const int nt = A.tp.n_tiles;
    const size_t rec = sizeof(TapeRec<Real>);
    const int wpb = BLOCK / 64;  // wavefronts per block
    size_t free_b = 0;
    char* pool = nullptr;
    // per buffer: tile_count[nt], bin_start[nt], tile_end[nt], overflow, wave_count[max_nw],
    // slice[nt][binning blocks]
    uint32_t* meta[REPLAY_BUFFERS] = {};
    unsigned long long* ctr1 = nullptr;  // counters of buffers 1.. (buffer 0 uses the caller's)
    DepositItem* ditems = nullptr;
    const int max_items = nt + DEP_ITEMS_PER_CU * n_cu + 1;
    std::vector<uint32_t> h_count(nt), h_bins(2 * (size_t)nt);
    std::vector<DepositItem> h_items;
    // pinned host copies per buffer: tile counts, overflow flag, wave counts, counters
    char* hpin[REPLAY_BUFFERS] = {};
    size_t hpin_bytes = 0, off_over = 0, off_wave = 0, off_ctr = 0;
    hipEvent_t ev_start = nullptr, counted[REPLAY_BUFFERS] = {}, deposited[REPLAY_BUFFERS] = {};
    hipEvent_t r0[REPLAY_BUFFERS] = {}, r1[REPLAY_BUFFERS] = {};
    std::vector<hipEvent_t> dep_ev;  // begin, end of every chunk's binning and deposits (timed calls)
    struct Slot {
        bool used = false;
        uint64_t start = 0, n = 0;
        int nw = 0;
    };
    Slot slot[REPLAY_BUFFERS];
    KArgs<Real> ka[REPLAY_BUFFERS];
    for (int b = 0; b < REPLAY_BUFFERS; ++b) ka[b] = A;
    std::vector<std::pair<uint64_t, uint64_t>> pending;  // ranges to replay again, smaller
    std::vector<int> order;                             // buffers in flight, in issue order
    uint64_t P = 0, r_cap = 0, b_cap = 0, next = 0, chunk = 0;
    const uint64_t chunk_max = std::max<uint64_t>(256, (n_photons + MIN_REPLAY_CHUNKS - 1) / MIN_REPLAY_CHUNKS);
    int max_nw = 0;
    const double hint = tape_hint(wkey);
    double max_rate = 0.0;
    float ms = 0.f;

    CHECK_HIP(available_bytes(&free_b));
    {
        const uint64_t lim = std::min<uint64_t>(free_b / 8 * 3, (uint64_t)96 << 30) / rec;
        P = std::max<uint64_t>(n_photons * 48, (uint64_t)1 << 20);
        if (hint > 0.0) P = std::max<uint64_t>(P, (uint64_t)std::min(5.8 * hint * (double)n_photons, 4.0e18));
        P = std::min<uint64_t>(P, lim);
        if (tape_limit > 0) P = std::min<uint64_t>(P, (uint64_t)tape_limit);
    }
    {
        // slots per photon: a wavefront slice 80% full at the busiest
        // wavefront's rays per photon, four and a half tile crossings per ray
        const double rays = hint > 0.0 ? hint / 0.8 : 80.0, bins = hint > 0.0 ? 4.5 * hint : 288.0;
        r_cap = (uint64_t)((double)P * rays / (REPLAY_BUFFERS * rays + bins));
        r_cap = std::min(std::max(r_cap, P / 16), P / 4 * 3 / REPLAY_BUFFERS);
        b_cap = P - REPLAY_BUFFERS * r_cap;
        // bin slots are 32-bit indices (at most 2^31 - 1 records), ray slots
        // are not: a large tape gives the excess back
        b_cap = std::min<uint64_t>(b_cap, ((uint64_t)1 << 31) - 1);
        r_cap = std::min<uint64_t>(r_cap, ((uint64_t)1 << 31) - 1);
        P = REPLAY_BUFFERS * r_cap + b_cap;
        // at least 64 slots per wavefront (fewer resident blocks if the tape is small)
        if (r_cap < 64 * (uint64_t)max_blocks * wpb) max_blocks = (int)(r_cap / (64 * (uint64_t)wpb));
        if (max_blocks < 1 || b_cap < 64) return TAPE_FALLBACK;
        chunk = (uint64_t)std::max(256.0, std::min((double)r_cap / rays, (double)b_cap / bins));
        chunk = std::min<uint64_t>(std::min<uint64_t>(n_photons, chunk), chunk_max);
    }
    max_nw = max_blocks * wpb;
    // pinned layout: tile counts [nt], overflow flag, (pad), wave counts [max_nw], counters [1 + ST_N]
    off_over = sizeof(uint32_t) * (size_t)nt;
    off_wave = sizeof(uint32_t) * ((size_t)nt + 2);
    off_ctr = (off_wave + sizeof(uint32_t) * (size_t)max_nw + 7) & ~(size_t)7;
    hpin_bytes = off_ctr + sizeof(unsigned long long) * (1 + ST_N);

    CHECK_HIP(buf_acquire(BUF_BINS, P * rec, stream, (void**)&pool));
    for (int b = 0; b < REPLAY_BUFFERS; ++b) {
        const size_t meta_words = 3 * (size_t)nt + 1 + (size_t)max_nw + (size_t)nt * bin_blocks_max(max_nw, n_cu);
        CHECK_HIP(lib_alloc((void**)&meta[b], sizeof(uint32_t) * meta_words, stream));
        CHECK_HIP(hipHostMalloc((void**)&hpin[b], hpin_bytes, hipHostMallocDefault));
        CHECK_HIP(hipEventCreateWithFlags(&counted[b], hipEventDisableTiming));
        CHECK_HIP(hipEventCreateWithFlags(&deposited[b], hipEventDisableTiming));
        if (t_transport) {
            CHECK_HIP(hipEventCreate(&r0[b]));
            CHECK_HIP(hipEventCreate(&r1[b]));
        }
    }
    CHECK_HIP(lib_alloc((void**)&ctr1, sizeof(unsigned long long) * (REPLAY_BUFFERS - 1) * (1 + ST_N), stream));
    CHECK_HIP(lib_alloc((void**)&ditems, sizeof(DepositItem) * max_items, stream));
    for (int b = 0; b < REPLAY_BUFFERS; ++b) {
        KArgs<Real>& a = ka[b];
        a.tp.rec = reinterpret_cast<TapeRec<Real>*>(pool) + (size_t)b * r_cap;
        a.tp.brec = reinterpret_cast<TapeRec<Real>*>(pool) + REPLAY_BUFFERS * r_cap;
        a.tp.tile_count = meta[b];
        a.tp.bin_start = meta[b] + nt;
        a.tp.tile_end = meta[b] + 2 * nt;
        a.tp.overflow = meta[b] + 3 * nt;
        a.tp.wave_count = meta[b] + 3 * nt + 1;
        a.tp.slice = meta[b] + 3 * nt + 1 + max_nw;
        a.work = b == 0 ? counters : ctr1 + (size_t)(b - 1) * (1 + ST_N);
        a.stats = a.work + 1;
        a.tp.scale_gw = 1;  // the replay writes C, the binning passes multiply by gw[pixel]
    }
    // the replay streams start after what the caller's stream holds (the
    // tape space's previous users, the allocations above)
    CHECK_HIP(hipEventCreateWithFlags(&ev_start, hipEventDisableTiming));
    CHECK_HIP(hipEventRecord(ev_start, stream));
    for (int b = 0; b < REPLAY_BUFFERS; ++b) CHECK_HIP(hipStreamWaitEvent(rs[b], ev_start, 0));

    {
#define TRY_HIP(expr)                          \
    do {                                       \
        hipError_t e_ = (expr);                \
        if (e_ != hipSuccess) return e_;       \
    } while (0)
        // replay the next range into buffer b and count its rays per tile
        auto issue = [&](int b) -> hipError_t {
            uint64_t st = 0, n = 0;
            if (!pending.empty()) {
                st = pending.back().first;
                n = pending.back().second;
                if (n > chunk) {
                    pending.back().first += chunk;
                    pending.back().second -= chunk;
                    n = chunk;
                } else {
                    pending.pop_back();
                }
            } else if (next < n_photons) {
                st = next;
                n = std::min<uint64_t>(chunk, n_photons - next);
                next += n;
            } else {
                return hipSuccess;  // nothing left: the buffer stays idle
            }
            Slot& S = slot[b];
            KArgs<Real>& a = ka[b];
            const hipStream_t s = rs[b];
            const int grid = (int)std::min<uint64_t>((n + BLOCK - 1) / BLOCK, (uint64_t)max_blocks);
            S.start = st;
            S.n = n;
            S.nw = grid * wpb;
            a.tp.rw = (uint32_t)std::min<uint64_t>(r_cap / S.nw, 0xffffffffu);
            a.tp.w0 = 0;
            a.tp.split = bin_split(S.nw, n_cu);
            a.tp.n_slices = S.nw * a.tp.split;
            a.pid0 = pid0 + st;
            a.n_photons = n;
            // the buffer's rays and counts are free once its last chunk is deposited
            if (S.used) TRY_HIP(hipStreamWaitEvent(s, deposited[b], 0));
            TRY_HIP(launch_fill_u32(a.tp.tile_count, nt, s));
            TRY_HIP(launch_fill_u32(a.tp.overflow, 1, s));
            TRY_HIP(launch_fill_u64(a.work, 1 + ST_N, s));
            if (r0[b]) TRY_HIP(hipEventRecord(r0[b], s));
            TRY_HIP(launch_transport<Real>(a, MODE_TAPE, TALLY_F64, grid, s));
            if (r1[b]) TRY_HIP(hipEventRecord(r1[b], s));
            TRY_HIP(launch_bin<Real>(a, false, s));
            char* h = hpin[b];
            TRY_HIP(hipMemcpyAsync(h, a.tp.tile_count, sizeof(uint32_t) * nt, hipMemcpyDeviceToHost, s));
            TRY_HIP(hipMemcpyAsync(h + off_over, a.tp.overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
            TRY_HIP(hipMemcpyAsync(h + off_wave, a.tp.wave_count, sizeof(uint32_t) * S.nw, hipMemcpyDeviceToHost, s));
            TRY_HIP(hipMemcpyAsync(h + off_ctr, a.work, sizeof(unsigned long long) * (1 + ST_N),
                                   hipMemcpyDeviceToHost, s));
            TRY_HIP(hipEventRecord(counted[b], s));
            S.used = true;
            order.push_back(b);
            return hipSuccess;
        };
#undef TRY_HIP
        for (int b = 0; b < REPLAY_BUFFERS; ++b) CHECK_HIP(issue(b));
        while (!order.empty()) {
            const int b = order.front();
            order.erase(order.begin());
            Slot& S = slot[b];
            CHECK_HIP(hipEventSynchronize(counted[b]));
            if (r0[b]) {
                CHECK_HIP(hipEventElapsedTime(&ms, r0[b], r1[b]));
                *t_transport += ms;
            }
            const char* h = hpin[b];
            const uint32_t* hc = reinterpret_cast<const uint32_t*>(h);
            const uint32_t h_over = *reinterpret_cast<const uint32_t*>(h + off_over);
            const uint32_t* hw = reinterpret_cast<const uint32_t*>(h + off_wave);
            const unsigned long long* hctr = reinterpret_cast<const unsigned long long*>(h + off_ctr);
            uint32_t busiest = 0;
            for (int w = 0; w < S.nw; ++w) busiest = std::max(busiest, hw[w]);
            const double rate = (double)busiest * S.nw / (double)S.n;  // rays per photon, busiest wavefront
            uint64_t crossings = 0;
            bool too_big = h_over != 0;
            for (int i = 0; i < nt; ++i) {
                crossings += hc[i];
                too_big = too_big || hc[i] > b_cap;
            }
            if (too_big) {
                // nothing of it reached the gradient: replay its range in halves
                if (S.n == 1) {
                    rc = MC_ERR_OUT_OF_MEMORY;
                    goto done;
                }
                pending.push_back({S.start, S.n});
                chunk = std::max<uint64_t>(1, S.n / 2);
                CHECK_HIP(issue(b));
                continue;
            }
            max_rate = std::max(max_rate, rate);
            for (int i = 1; i < 1 + ST_N; ++i) host_sum[i] += hctr[i];
            std::copy(hc, hc + nt, h_count.begin());
            // the host arrays of the previous chunk's deposits must have been read
            CHECK_HIP(hipStreamSynchronize(stream));
            if (t_tape) {
                hipEvent_t e0 = nullptr, e1 = nullptr;
                CHECK_HIP(hipEventCreate(&e0));
                dep_ev.push_back(e0);
                CHECK_HIP(hipEventCreate(&e1));
                dep_ev.push_back(e1);
                CHECK_HIP(hipEventRecord(e0, stream));
            }
            rc = deposit_groups<Real>(ka[b], tally, h_count, b_cap, n_cu, ditems, max_items, h_bins, h_items, stream);
            if (rc != MC_OK) goto done;
            if (t_tape) CHECK_HIP(hipEventRecord(dep_ev.back(), stream));
            CHECK_HIP(hipEventRecord(deposited[b], stream));
            // next chunk: the busiest wavefront's slice about 80% full and the
            // crossings (with 5% to spare) in the bin space
            if (rate > 0.0) {
                const double rays = rate / 0.8, bins = 1.05 * (double)crossings / (double)S.n;
                double nx = std::floor((double)r_cap / rays);
                if (bins > 0.0) nx = std::min(nx, std::floor((double)b_cap / bins));
                chunk = std::min<uint64_t>((uint64_t)std::max(1.0, nx), chunk_max);
            }
            CHECK_HIP(issue(b));
        }
    }
    CHECK_HIP(hipStreamSynchronize(stream));
    for (size_t i = 0; i + 1 < dep_ev.size(); i += 2) {
        CHECK_HIP(hipEventElapsedTime(&ms, dep_ev[i], dep_ev[i + 1]));
        *t_tape += ms;
    }
    // (chunks of very few photons measure noisy rates: only large calls set the hint)
    if (n_photons >= 65536) set_tape_hint(wkey, max_rate);

done:
    // nothing may still run on the replay streams when the buffers are released
    for (int b = 0; b < REPLAY_BUFFERS; ++b) (void)hipStreamSynchronize(rs[b]);
    {
        std::vector<void*> bufs = {(void*)ditems, (void*)ctr1};
        for (int b = 0; b < REPLAY_BUFFERS; ++b) bufs.push_back((void*)meta[b]);
        for (void* p : bufs) {
            if (!p) continue;
            hipError_t e = hipFreeAsync(p, stream);
            if (rc == MC_OK && e != hipSuccess) rc = map_err(e);
        }
    }
    if (pool) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        buf_release(dev, BUF_BINS, pool, stream);
    }
    // the host arrays above were sources or targets of asynchronous copies
    (void)hipStreamSynchronize(stream);
    for (int b = 0; b < REPLAY_BUFFERS; ++b) {
        if (hpin[b]) (void)hipHostFree(hpin[b]);
        for (hipEvent_t e : {counted[b], deposited[b], r0[b], r1[b]})
            if (e) (void)hipEventDestroy(e);
    }
    if (ev_start) (void)hipEventDestroy(ev_start);
    for (hipEvent_t e : dep_ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

template <typename Real>
int run_tape(KArgs<Real> A, int tally, uint64_t n_photons, uint64_t pid0, int64_t tape_limit, int max_blocks,
             int n_cu, unsigned long long* counters, unsigned long long* host_sum, double* t_transport,
             double* t_tape, hipStream_t stream, uint64_t wkey, const MixPath* mp = nullptr) {
    if (!mp) {
        hipStream_t rs[REPLAY_BUFFERS];
        if (replay_streams(rs))
            return run_tape_overlap<Real>(A, tally, n_photons, pid0, tape_limit, max_blocks, n_cu, counters,
                                          host_sum, t_transport, t_tape, stream, wkey, rs);
    }
    int rc = MC_OK;
    // device times: replay (r0, r1), binning + deposit of the last chunk (b0, b1)
    hipEvent_t r0 = nullptr, r1 = nullptr, b0 = nullptr, b1 = nullptr;
    bool pending_b = false;
    float ms = 0.f;
    const int nt = A.tp.n_tiles;
    const size_t rec = sizeof(TapeRec<Real>);
    const int wpb = BLOCK / 64;  // wavefronts per block
    size_t free_b = 0;
    char* pool = nullptr;
    // tile_count[nt], bin_start[nt], tile_end[nt], overflow, wave_count[max_nw], slice[nt][binning blocks]
    uint32_t* meta = nullptr;
    DepositItem* ditems = nullptr;
    const int max_items = nt + DEP_ITEMS_PER_CU * n_cu + 1;
    std::vector<uint32_t> h_count(nt), h_bins(2 * (size_t)nt);
    std::vector<uint32_t> h_wave;
    std::vector<DepositItem> h_items;
    unsigned long long h_ctr[1 + ST_N];
    uint32_t h_over = 0;
    uint64_t P = 0, r_cap = 0, r_min = 0, done = 0, chunk = 0;
    int max_nw = 0;
    const double hint = tape_hint(wkey);
    double max_rate = 0.0;

    CHECK_HIP(available_bytes(&free_b));
    {
        // (slots are 32-bit indices: at most 2^31 - 1 records)
        const uint64_t lim = std::min<uint64_t>(free_b / 8 * 3, (uint64_t)96 << 30) / rec;
        P = std::max<uint64_t>(n_photons * 48, (uint64_t)1 << 20);
        // a workload measured before gets room for all its rays and their
        // bins at once where memory allows: every chunk is a launch of the
        // replay with its own tail (the last, longest photons)
        if (hint > 0.0) P = std::max<uint64_t>(P, (uint64_t)std::min(5.8 * hint * (double)n_photons, 4.0e18));
        P = std::min<uint64_t>(std::min<uint64_t>(P, lim), ((uint64_t)1 << 31) - 1);
        if (tape_limit > 0) P = std::min<uint64_t>(P, (uint64_t)tape_limit);
    }
    // the rays get between an eighth and seven eighths of the space, and at
    // least 64 slots per wavefront (fewer resident blocks if the tape is small)
    r_min = P / 8;
    if (r_min < 64 * (uint64_t)max_blocks * wpb) max_blocks = (int)(r_min / (64 * (uint64_t)wpb));
    if (max_blocks < 1 || P - r_min < 64) return TAPE_FALLBACK;
    max_nw = max_blocks * wpb;
    h_wave.resize(max_nw);
    r_cap = P / 2;

    if (t_transport) {
        CHECK_HIP(hipEventCreate(&r0));
        CHECK_HIP(hipEventCreate(&r1));
        CHECK_HIP(hipEventCreate(&b0));
        CHECK_HIP(hipEventCreate(&b1));
    }
    CHECK_HIP(buf_acquire(BUF_BINS, P * rec, stream, (void**)&pool));
    {
        const size_t meta_words = 3 * (size_t)nt + 1 + (size_t)max_nw + (size_t)nt * bin_blocks_max(max_nw, n_cu);
        CHECK_HIP(lib_alloc((void**)&meta, sizeof(uint32_t) * meta_words, stream));
    }
    CHECK_HIP(lib_alloc((void**)&ditems, sizeof(DepositItem) * max_items, stream));
    A.tp.rec = reinterpret_cast<TapeRec<Real>*>(pool);
    A.tp.tile_count = meta;
    A.tp.bin_start = meta + nt;
    A.tp.tile_end = meta + 2 * nt;
    A.tp.overflow = meta + 3 * nt;
    A.tp.wave_count = meta + 3 * nt + 1;
    A.tp.slice = meta + 3 * nt + 1 + max_nw;
    // the replay writes C and the binning passes multiply by gw[pixel], except
    // for a mixture's full gradient, whose replay sums gw C per collision
    A.tp.scale_gw = mp ? 0 : 1;

    if (mp) {
        A.mix_rows = mp->rows;
        A.mix_evcap = mp->cap;
    }
    // first chunk: from the rays per photon measured on this workload before
    // (busiest wavefront, with a fifth to spare, and four tile crossings per
    // ray for the bins), else a guess of 64 rays per photon
    if (hint > 0.0)
        chunk = (uint64_t)std::max(256.0, std::min(0.8 * (double)r_cap / hint, (double)(P - r_cap) / (4.5 * hint)));
    else
        chunk = std::max<uint64_t>(256, r_cap / 64);
    chunk = std::min<uint64_t>(n_photons, chunk);
    while (done < n_photons) {
        if (mp) chunk = std::min<uint64_t>(chunk, mp->max_chunk);
        const uint64_t n = std::min<uint64_t>(chunk, n_photons - done);
        const uint64_t b_cap = P - r_cap;
        const int grid = (int)std::min<uint64_t>((n + BLOCK - 1) / BLOCK, (uint64_t)max_blocks);
        const int nw = grid * wpb;
        A.tp.rw = (uint32_t)std::min<uint64_t>(r_cap / nw, 0xffffffffu);
        A.tp.brec = reinterpret_cast<TapeRec<Real>*>(pool) + r_cap;
        A.tp.w0 = 0;
        A.tp.split = bin_split(nw, n_cu);
        A.tp.n_slices = nw * A.tp.split;
        A.pid0 = pid0 + done;
        A.n_photons = n;
        CHECK_HIP(launch_fill_u32(A.tp.tile_count, nt, stream));
        CHECK_HIP(launch_fill_u32(A.tp.overflow, 1, stream));
        CHECK_HIP(launch_fill_u64(counters, 1 + ST_N, stream));
        if (mp) CHECK_HIP(launch_fill_f64(mp->rows, (int64_t)(n * (mp->cap + 1)), stream));
        if (r0) CHECK_HIP(hipEventRecord(r0, stream));
        CHECK_HIP(launch_transport<Real>(A, MODE_TAPE, TALLY_F64, grid, stream));
        if (r1) CHECK_HIP(hipEventRecord(r1, stream));
        CHECK_HIP(launch_bin<Real>(A, false, stream));
        CHECK_HIP(hipMemcpyAsync(h_count.data(), A.tp.tile_count, sizeof(uint32_t) * nt, hipMemcpyDeviceToHost,
                                 stream));
        CHECK_HIP(hipMemcpyAsync(&h_over, A.tp.overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
        CHECK_HIP(hipMemcpyAsync(h_wave.data(), A.tp.wave_count, sizeof(uint32_t) * nw, hipMemcpyDeviceToHost,
                                 stream));
        CHECK_HIP(hipMemcpyAsync(h_ctr, counters, sizeof(h_ctr), hipMemcpyDeviceToHost, stream));
        CHECK_HIP(hipStreamSynchronize(stream));
        if (r0) {
            CHECK_HIP(hipEventElapsedTime(&ms, r0, r1));
            *t_transport += ms;
            if (pending_b) {
                CHECK_HIP(hipEventElapsedTime(&ms, b0, b1));
                *t_tape += ms;
                pending_b = false;
            }
        }
        uint32_t busiest = 0;
        for (int w = 0; w < nw; ++w) busiest = std::max(busiest, h_wave[w]);
        const double rate = (double)busiest * nw / (double)n;  // rays per photon, busiest wavefront
        max_rate = std::max(max_rate, rate);
        uint64_t crossings = 0;
        bool too_big = h_over != 0;
        for (int i = 0; i < nt; ++i) {
            crossings += h_count[i];
            too_big = too_big || h_count[i] > b_cap;
        }
        if (too_big) {
            if (n == 1) {
                rc = MC_ERR_OUT_OF_MEMORY;
                goto done;
            }
            chunk = n / 2;
            continue;
        }
        for (int i = 1; i < 1 + ST_N; ++i) host_sum[i] += h_ctr[i];
        if (b0) CHECK_HIP(hipEventRecord(b0, stream));
        rc = deposit_groups<Real>(A, tally, h_count, b_cap, n_cu, ditems, max_items, h_bins, h_items, stream);
        if (rc != MC_OK) goto done;
        if (mp) CHECK_HIP(launch_mix_path<Real>(A, mp->grid, stream));
        if (b1) {
            CHECK_HIP(hipEventRecord(b1, stream));
            pending_b = true;
        }
        done += n;
        // next chunk: the busiest wavefront's slice about 80% full and the
        // crossings (with 5% to spare) in the bin space
        if (rate > 0.0) {
            const double rays = rate / 0.8, bins = 1.05 * (double)crossings / (double)n;
            const double fit = std::floor((double)P / (rays + bins));
            r_cap = (uint64_t)std::ceil(std::max(1.0, fit) * rays);
            r_cap = std::min(std::max(r_cap, r_min), P - r_min);
            double next = std::floor((double)r_cap / rays);
            if (bins > 0.0) next = std::min(next, std::floor((double)(P - r_cap) / bins));
            chunk = (uint64_t)std::max(1.0, next);
        } else {
            chunk = n_photons - done;
        }
    }
    CHECK_HIP(hipStreamSynchronize(stream));
    if (pending_b) {
        CHECK_HIP(hipEventElapsedTime(&ms, b0, b1));
        *t_tape += ms;
    }
    // (chunks of very few photons measure noisy rates: only large calls set the hint)
    if (n_photons >= 65536) set_tape_hint(wkey, max_rate);

done:
    for (void* p : {(void*)ditems, (void*)meta}) {
        if (!p) continue;
        hipError_t e = hipFreeAsync(p, stream);
        if (rc == MC_OK && e != hipSuccess) rc = map_err(e);
    }
    {
        int dev = 0;
        (void)hipGetDevice(&dev);
        buf_release(dev, BUF_BINS, pool, stream);
    }
    // the host arrays above were sources of asynchronous copies
    (void)hipStreamSynchronize(stream);
    for (hipEvent_t e : {r0, r1, b0, b1})
        if (e) (void)hipEventDestroy(e);
    return rc;
}

constexpr uint32_t TAPE_MAGIC = 0x6d637470u;

uint64_t camera_hash(int n_cams, const mc_camera* cams) {
    uint64_t h = 1469598103934665603ull;
    const unsigned char* b = reinterpret_cast<const unsigned char*>(cams);
    for (size_t i = 0; i < sizeof(mc_camera) * (size_t)n_cams; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

// Key of a workload for the tape sizing hint: the grid, the cameras and the
// parameters that shape the photon paths (not the photon count or seed).
uint64_t workload_key(const mc_grid* g, int n_cams, const mc_camera* cams, const mc_params* p) {
    uint64_t h = camera_hash(n_cams, cams);
    const double v[10] = {(double)g->nx, (double)g->ny, (double)g->nz, g->dx, g->dy, g->dz,
                          p->albedo, p->g, p->sun_zenith, p->sun_azimuth};
    const unsigned char* b = reinterpret_cast<const unsigned char*>(v);
    for (size_t i = 0; i < sizeof(v); ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

// Gradient of a large grid from the rays a render kept: the record weights
// are local estimates, scaled by the pixel weights in the binning passes;
// the slices are binned and deposited in passes whose tile crossings fit
// the bin space (crossings per ray estimated from the passes so far).
template <typename Real>
int run_tape_kept(KArgs<Real> A, int tally, const mc_tape* T, int64_t tape_limit, int n_cu, double* t_tape,
                  hipStream_t stream, int scale_gw = 1) {
    int rc = MC_OK;
    hipEvent_t b0 = nullptr, b1 = nullptr;
    float ms = 0.f;
    const int nt = A.tp.n_tiles;
    const size_t rec = sizeof(TapeRec<Real>);
    size_t free_b = 0;
    char* pool = nullptr;
    uint32_t* meta = nullptr;  // tile_count[nt], bin_start[nt], tile_end[nt], slice[nt][binning blocks]
    DepositItem* ditems = nullptr;
    const int max_items = nt + DEP_ITEMS_PER_CU * n_cu + 1;
    std::vector<uint32_t> h_count(nt), h_bins(2 * (size_t)nt);
    std::vector<uint32_t> h_wave((size_t)T->nw);
    std::vector<DepositItem> h_items;
    uint64_t P = 0;
    double per_ray = 4.0;  // tile crossings per ray (first guess)
    int w0 = 0;

    CHECK_HIP(available_bytes(&free_b));
    P = std::min<uint64_t>(free_b / 4, (uint64_t)32 << 30) / rec;
    P = std::min<uint64_t>(P, ((uint64_t)1 << 31) - 1);
    if (tape_limit > 0) P = std::min<uint64_t>(P, (uint64_t)tape_limit);
    if (P < 64) return MC_ERR_OUT_OF_MEMORY;
    CHECK_HIP(hipEventCreate(&b0));
    CHECK_HIP(hipEventCreate(&b1));
    CHECK_HIP(buf_acquire(BUF_BINS, P * rec, stream, (void**)&pool));
    {
        const size_t meta_words = 3 * (size_t)nt + (size_t)nt * bin_blocks_max(T->nw, n_cu);
        CHECK_HIP(lib_alloc((void**)&meta, sizeof(uint32_t) * meta_words, stream));
    }
    CHECK_HIP(lib_alloc((void**)&ditems, sizeof(DepositItem) * max_items, stream));
    CHECK_HIP(hipMemcpyAsync(h_wave.data(), T->wave_count, sizeof(uint32_t) * T->nw, hipMemcpyDeviceToHost,
                             stream));
    A.tp.rec = reinterpret_cast<TapeRec<Real>*>(T->rec);
    A.tp.rw = T->rw;
    A.tp.wave_count = T->wave_count;
    A.tp.scale_gw = scale_gw;
    A.tp.brec = reinterpret_cast<TapeRec<Real>*>(pool);
    A.tp.tile_count = meta;
    A.tp.bin_start = meta + nt;
    A.tp.tile_end = meta + 2 * nt;
    A.tp.slice = meta + 3 * nt;
    CHECK_HIP(hipEventRecord(b0, stream));
    CHECK_HIP(hipStreamSynchronize(stream));  // h_wave
    while (w0 < T->nw) {
        // the slices whose estimated crossings fit the bin space
        int ns = 0;
        double rays = 0.0;
        while (w0 + ns < T->nw) {
            const double r = (double)std::min(h_wave[w0 + ns], T->rw);
            if (ns > 0 && (rays + r) * per_ray * 1.05 > (double)P) break;
            rays += r;
            ++ns;
        }
        A.tp.w0 = w0;
        A.tp.split = bin_split(ns, n_cu);
        A.tp.n_slices = ns * A.tp.split;
        CHECK_HIP(launch_fill_u32(A.tp.tile_count, nt, stream));
        CHECK_HIP(launch_bin<Real>(A, false, stream));
        CHECK_HIP(hipMemcpyAsync(h_count.data(), A.tp.tile_count, sizeof(uint32_t) * nt, hipMemcpyDeviceToHost,
                                 stream));
        CHECK_HIP(hipStreamSynchronize(stream));
        uint64_t crossings = 0;
        bool too_big = false;
        for (int i = 0; i < nt; ++i) {
            crossings += h_count[i];
            too_big = too_big || h_count[i] > P;
        }
        if (too_big) {
            if (ns == 1) {
                rc = MC_ERR_OUT_OF_MEMORY;
                goto done;
            }
            per_ray = std::max(2.0 * per_ray, (double)crossings / std::max(rays, 1.0));
            continue;
        }
        rc = deposit_groups<Real>(A, tally, h_count, P, n_cu, ditems, max_items, h_bins, h_items, stream);
        if (rc != MC_OK) goto done;
        if (rays > 0.0) per_ray = std::max(1.0, (double)crossings / rays);
        w0 += ns;
    }
    CHECK_HIP(hipEventRecord(b1, stream));
    CHECK_HIP(hipStreamSynchronize(stream));
    CHECK_HIP(hipEventElapsedTime(&ms, b0, b1));
    if (t_tape) *t_tape += ms;

done:
    for (void* p : {(void*)ditems, (void*)meta}) {
        if (!p) continue;
        hipError_t e = hipFreeAsync(p, stream);
        if (rc == MC_OK && e != hipSuccess) rc = map_err(e);
    }
    {
        int dev = 0;
        (void)hipGetDevice(&dev);
        buf_release(dev, BUF_BINS, pool, stream);
    }
    (void)hipStreamSynchronize(stream);
    for (hipEvent_t e : {b0, b1})
        if (e) (void)hipEventDestroy(e);
    return rc;
}

// Releases a tape's device memory (stream-ordered) and the tape.
void tape_release(mc_tape* t, hipStream_t stream) {
    if (!t) return;
    buf_release(t->device, BUF_TAPE, t->rec, stream);
    if (t->wave_count) (void)hipFreeAsync(t->wave_count, stream);
    t->magic = 0;
    delete t;
}

// One call of the transport kernel with all its preparation.
// Gradient of a mixture: k_mix_grad over the photons in chunks; each chunk's
// connection terms go to per-wavefront record slices, binned by tile and
// deposited in LDS (run_tape_kept on the slices, weights already final);
// records that do not fit a slice, and grids without tiles, deposit with
// device atomics in the kernel.
template <typename Real>
int run_mixgrad(KArgs<Real> A, const mc_params* prm, int grid_blocks, int n_cu, double* t_tape, hipStream_t stream) {
    int rc = MC_OK;
    const int nw = grid_blocks * (BLOCK / 64);
    void* rec = nullptr;
    uint32_t* wc = nullptr;
    double* evs = nullptr;
    uint64_t rw = 0, chunk = prm->n_photons;
    if (A.tape) {
        // records: sized for 16 local estimates per photon (cloud scenes have
        // about that many) with half again as margin per slice, in chunks of
        // photons whose records fit a quarter of the free memory (at most
        // 16 GiB); a slice that still fills up deposits the rest directly
        size_t avail = 0;
        CHECK_HIP(available_bytes(&avail));
        const double per_photon = 16.0;
        uint64_t cap = std::min<uint64_t>(avail / 4, (uint64_t)16 << 30) / sizeof(TapeRec<Real>);
        if (prm->tape_limit > 0) cap = std::min<uint64_t>(cap, (uint64_t)prm->tape_limit);
        chunk = std::min<uint64_t>(prm->n_photons, (uint64_t)(0.66 * (double)cap / per_photon));
        rw = std::min<uint64_t>((uint64_t)(1.5 * per_photon * (double)chunk / nw) + 64,
                                std::min<uint64_t>(cap / nw, 0xffffffffull / nw));
        if (chunk == 0 || rw < 64 || lib_alloc(&rec, sizeof(TapeRec<Real>) * rw * nw, stream) != hipSuccess ||
            lib_alloc((void**)&wc, sizeof(uint32_t) * (nw + 1), stream) != hipSuccess) {
            (void)hipGetLastError();
            A.tape = 0;
            chunk = prm->n_photons;
        } else {
            A.tp.rec = reinterpret_cast<TapeRec<Real>*>(rec);
            A.tp.rw = (uint32_t)rw;
            A.tp.wave_count = wc;
        }
    }
    if (A.mix_full) {
        // the full gradient's second pass reads the first collisions' sums
        // of the first pass instead of walking their estimates again
        const uint32_t cap = 32;
        if (lib_alloc((void**)&evs, sizeof(double) * cap * (size_t)grid_blocks * BLOCK, stream) == hipSuccess) {
            A.mix_evs = evs;
            A.mix_evcap = cap;
        } else {
            (void)hipGetLastError();
        }
    }
    for (uint64_t done = 0; done < prm->n_photons; done += chunk) {
        A.pid0 = prm->photon_offset + done;
        A.n_photons = std::min<uint64_t>(chunk, prm->n_photons - done);
        if (A.tape) CHECK_HIP(launch_fill_u32(wc, nw + 1, stream));
        CHECK_HIP(launch_transport<Real>(A, MODE_MIXGRAD, TALLY_F64, grid_blocks, stream));
        if (A.tape) {
            mc_tape T;
            T.rec = rec;
            T.wave_count = wc;
            T.nw = nw;
            T.rw = (uint32_t)rw;
            rc = run_tape_kept<Real>(A, TALLY_F64, &T, 0, n_cu, t_tape, stream, 0);
            if (rc != MC_OK) goto done;
        }
    }
done:
    for (void* p : {rec, (void*)wc, (void*)evs}) {
        if (!p) continue;
        hipError_t e = hipFreeAsync(p, stream);
        if (rc == MC_OK && e != hipSuccess) rc = map_err(e);
    }
    return rc;
}

template <typename Real>
int run(int mode, const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
        const mc_params* prm, double* images, double* images_m2, const double* dl, double* grad, mc_stats* stats,
        uint64_t first_pid, uint32_t trace_count, uint32_t max_rec, mc_event* ev, int32_t* pix,
        mc_path* paths, hipStream_t stream, mc_tape** keep = nullptr, const mc_tape* src = nullptr,
        uint32_t n_pp = 0, const MixIn* mix = nullptr, const void* beta_eval = nullptr,
        void* fixed_scratch = nullptr, CaptureArgs* cap = nullptr) {
    // fixed_scratch: the no-allocation render; its scratch is the library's
    // fixed device array (NOALLOC_SCRATCH_BYTES) and the call allocates
    // nothing and creates no events
    int rc = MC_OK;
    const int64_t n_pix = pixel_count(n_cams, cams);
    const int64_t n_vox = (int64_t)grid->nx * grid->ny * grid->nz;
    const int tally = prm->tally == MC_TALLY_KAHAN32 ? TALLY_K32 : TALLY_F64;
    const bool k32 = tally == TALLY_K32 && mode != MODE_TRACE && mode != MODE_VOXEL && mode != MODE_MIXGRAD;

    // occupancy mask: one bit per run of 2^msh consecutive voxels, the
    // shortest runs whose bits fit the kernels' LDS copy (the FP32 budget for
    // the mixed-precision render, which runs four blocks per CU as FP32 does)
    const bool mixed_render = prm->transport == MC_MIXED && mode == MODE_RENDER;
    const int64_t mask_budget = sizeof(Real) == 4 || mixed_render ? MASK_WORDS_FP32 : MASK_WORDS;
    int msh = 0;
    while (((n_vox + ((int64_t)1 << msh) - 1) >> msh) > mask_budget * 32) ++msh;
    const int64_t mask_words = (((n_vox + ((int64_t)1 << msh) - 1) >> msh) + 31) / 32;

    // mixed precision: the photons in FP64 (Real = double), the connection
    // rays on a float copy of beta
    const bool mixed = sizeof(Real) == 8 && prm->transport == MC_MIXED && mode == MODE_RENDER && !mix && !beta_eval;
    size_t bytes = round256(sizeof(unsigned long long) * (1 + ST_N)) +
                   round256(sizeof(Real) * (n_vox + BETA_PAD + grid->nz)) * (beta_eval ? 2 : 1) +
                   round256(sizeof(uint32_t)) +
                   round256(sizeof(DevCam<Real>) * n_cams) + round256(sizeof(NormCam) * n_cams) +
                   round256(sizeof(uint32_t) * mask_words);
    if (mode == MODE_GRAD || mode == MODE_MIXGRAD) bytes += round256(sizeof(double) * n_pix);
    if (mixed) bytes += round256(sizeof(float) * (n_vox + BETA_PAD + grid->nz));
    if (k32 && mode == MODE_RENDER) bytes += round256(sizeof(float) * 2 * n_pix);
    if (k32 && mode == MODE_GRAD) bytes += round256(sizeof(float) * 2 * n_vox);
    if (mode == MODE_BMC) bytes += round256(sizeof(HostCam) * n_cams);
    // voxel model: the tally L, [voxel][cameras rounded up to a multiple of 8]
    const int lc_pitch = (n_cams + 7) & ~7;
    if (mode == MODE_VOXEL) bytes += round256(sizeof(double) * n_vox * lc_pitch);
    bytes += 256;

    Scratch S;
    KArgs<Real> A;
    std::memset(&A, 0, sizeof(A));
    unsigned long long* counters = nullptr;
    Real* betap = nullptr;
    DevCam<Real>* dcams = nullptr;
    NormCam* ncams = nullptr;
    unsigned long long host_counters[1 + ST_N];
    double base_norm = 0.0;
    int dev = 0, n_cu = 0, per_cu = 0, grid_blocks = 1;
    const uint64_t n_norm = prm->n_photons_norm ? prm->n_photons_norm : prm->n_photons;
    // packets of the backward method: n_pp per pixel
    const uint64_t n_work = mode == MODE_BMC ? (uint64_t)n_pix * n_pp : prm->n_photons;
    const int64_t need_blocks = (int64_t)((n_work + BLOCK - 1) / BLOCK);
    bool tape_counts = false;
    bool mix_tape = false;  // a mixture's gradient by the queued tape replay
    uint64_t tape_key = 0;  // workload key of the tape sizing hint
    double* mix_rows = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;  // around the transport launch (stats only)
    double t_transport = 0.0, t_tape = 0.0;
    // a render that keeps its rays (only where the gradient would use tiles)
    mc_tape* kt = nullptr;
    bool keep_rays = false;
    int launch_mode = mode;
    if (keep) *keep = nullptr;

    CHECK_HIP(hipGetDevice(&dev));
    CHECK_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    if (fixed_scratch) {
        if (bytes > NOALLOC_SCRATCH_BYTES) return MC_ERR_SCRATCH_LIMIT;  // nothing enqueued yet
        S.base = static_cast<char*>(fixed_scratch);
    } else {
        CHECK_HIP(lib_alloc((void**)&S.base, bytes, stream));
    }
    counters = S.take<unsigned long long>(1 + ST_N);
    // beta, the zeros, then the air column of a mixture (one value per layer)
    betap = S.take<Real>(n_vox + BETA_PAD + grid->nz);
    A.beta_le = betap;
    if (beta_eval) {
        // frozen-event render: the local estimates walk a copy of beta_eval
        Real* bl = S.take<Real>(n_vox + BETA_PAD + grid->nz);
        CHECK_HIP(hipMemcpyAsync(bl, beta_eval, sizeof(Real) * n_vox, hipMemcpyDeviceToDevice, stream));
        if (sizeof(Real) == 4)
            CHECK_HIP(launch_fill_f32(reinterpret_cast<float*>(bl) + n_vox, BETA_PAD, stream));
        else
            CHECK_HIP(launch_fill_f64(reinterpret_cast<double*>(bl) + n_vox, BETA_PAD, stream));
        A.beta_le = bl;
        A.frozen = 1;
    }
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
    // the kernels read a copy of beta followed by zeros (an empty voxel
    // fetches beta[n_vox])
    A.air_base = (uint32_t)n_vox;
    A.air_step = 0;
    if (mix) {
        // a mixture: beta = air + sig * aer; when the air depends on the
        // height only, empty runs (of aerosol) read the air column
        CHECK_HIP(launch_mix_total<Real>(betap, mix->air, mix->aer, mix->sig, n_vox, BETA_PAD, stream));
        A.mix_air = mix->air;
        A.mix_aer = mix->aer;
        A.mix_sig = mix->sig;
        A.mix_full = mix->full;
        // (the gradient replays the same walks when its rays fit the tile
        // bins; the kernels that walk every photon alone read the full copy
        // of beta whatever the flag says)
        if (mode == MODE_RENDER || mode == MODE_MIXGRAD) {
            uint32_t* flag = S.take<uint32_t>(1);
            uint32_t h_flag = 1;
            CHECK_HIP(launch_fill_u32(flag, 1, stream));
            CHECK_HIP(launch_air_column<Real>(mix->air, n_vox, (int64_t)grid->nx * grid->ny, grid->nz,
                                              betap + n_vox + BETA_PAD, flag, stream));
            CHECK_HIP(hipMemcpyAsync(&h_flag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
            CHECK_HIP(hipStreamSynchronize(stream));
            if (h_flag == 0) {
                A.air_base = (uint32_t)(n_vox + BETA_PAD);
                A.air_step = 1;
            }
        }
    } else {
        CHECK_HIP(hipMemcpyAsync(betap, beta, sizeof(Real) * n_vox, hipMemcpyDeviceToDevice, stream));
        if (sizeof(Real) == 4)
            CHECK_HIP(launch_fill_f32(reinterpret_cast<float*>(betap) + n_vox, BETA_PAD, stream));
        else
            CHECK_HIP(launch_fill_f64(reinterpret_cast<double*>(betap) + n_vox, BETA_PAD, stream));
    }

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
    A.G.ddx = grid->dx;
    A.G.ddy = grid->dy;
    A.G.ddz = grid->dz;
    A.beta = betap;
    if (mixed) {
        float* bw = S.take<float>(n_vox + BETA_PAD + grid->nz);
        CHECK_HIP(launch_d2f(n_vox + BETA_PAD, reinterpret_cast<const double*>(betap), bw, stream));
        A.walk32 = 1;
        A.beta_w32 = bw;
        A.G32.nx = grid->nx;
        A.G32.ny = grid->ny;
        A.G32.nz = grid->nz;
        A.G32.nxy = grid->nx * grid->ny;
        A.G32.dx = (float)grid->dx;
        A.G32.dy = (float)grid->dy;
        A.G32.dz = (float)grid->dz;
        A.G32.idx = (float)(1.0 / grid->dx);
        A.G32.idy = (float)(1.0 / grid->dy);
        A.G32.idz = (float)(1.0 / grid->dz);
        A.G32.ddx = grid->dx;
        A.G32.ddy = grid->dy;
        A.G32.ddz = grid->dz;
    }
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
    A.msh = msh;
    A.mask_words = (int)mask_words;
    // the walks' buffer spans the voxels in the walk's precision: its byte
    // range stays below 2^31; larger grids (and MC_PLAIN_WALK_LOADS=1) take
    // plain loads
    A.walk_buf = (uint64_t)n_vox * (A.walk32 ? sizeof(float) : sizeof(Real)) < ((uint64_t)1 << 31) &&
                 !plain_walk_loads();
    {
        const bool lds_fits =
            ((mask_words + 1) & ~(int64_t)1) * 4 + n_vox * (int64_t)sizeof(double) <= GRAD_LDS_BYTES;
        A.grad_lds = mode == MODE_GRAD && lds_fits;
        keep_rays = mode == MODE_RENDER && keep && !lds_fits && prm->n_photons > 0;
    }
    if ((mode == MODE_GRAD && !A.grad_lds) || keep_rays || mode == MODE_MIXGRAD) {
        int shx, shy, shz;
        tape_tiles(grid, shx, shy, shz);
        const int tx = 1 << shx, ty = 1 << shy, tz = 1 << shz;
        const int ntx = (grid->nx + tx - 1) / tx, nty = (grid->ny + ty - 1) / ty, ntz = (grid->nz + tz - 1) / tz;
        if ((int64_t)ntx * nty * ntz <= MAX_TAPE_TILES) {
            A.tape = 1;
            A.tp.shx = shx;
            A.tp.shy = shy;
            A.tp.shz = shz;
            A.tp.n_tiles = ntx * nty * ntz;
            A.tp.itx = (Real)(1.0 / tx);
            A.tp.ity = (Real)(1.0 / ty);
            A.tp.itz = (Real)(1.0 / tz);
            A.tp.T.nx = ntx;
            A.tp.T.ny = nty;
            A.tp.T.nz = ntz;
            A.tp.T.nxy = ntx * nty;
            A.tp.T.dx = (Real)(grid->dx * tx);
            A.tp.T.dy = (Real)(grid->dy * ty);
            A.tp.T.dz = (Real)(grid->dz * tz);
            A.tp.T.idx = (Real)(1.0 / (grid->dx * tx));
            A.tp.T.idy = (Real)(1.0 / (grid->dy * ty));
            A.tp.T.idz = (Real)(1.0 / (grid->dz * tz));
        }
    }
    if (keep_rays && !A.tape) keep_rays = false;  // too many tiles: the gradient replays
    if (keep_rays) {
        A.tape = 0;  // the render itself runs in one launch
        launch_mode = MODE_RTAPE;
    }
    mix_tape = mode == MODE_MIXGRAD && A.tape;
    CHECK_HIP(transport_occupancy<Real>(A, A.tape && (mode != MODE_MIXGRAD || mix_tape) ? MODE_TAPE : launch_mode,
                                        tally, &per_cu));
    if (mode != MODE_TRACE) {
        uint32_t* mask = S.take<uint32_t>(mask_words);
        A.mask = mask;
        if (A.air_step)
            CHECK_HIP(launch_build_mask_aer<Real>(A, mask, stream));
        else
            CHECK_HIP(launch_build_mask<Real>(A, mask, stream));
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
    } else if (mode == MODE_BMC) {
        A.img = images;
        A.img_m2 = images_m2;
        A.n_pp = n_pp;
        CHECK_HIP(launch_fill_f64(images, n_pix, stream));
        if (images_m2) CHECK_HIP(launch_fill_f64(images_m2, n_pix, stream));
        HostCam* hc = S.take<HostCam>(n_cams);
        int64_t off = 0;
        for (int first = 0; first < n_cams; first += CAM_CHUNK) {
            CamChunk ch;
            std::memset(&ch, 0, sizeof(ch));
            ch.first = first;
            ch.n = n_cams - first < CAM_CHUNK ? n_cams - first : CAM_CHUNK;
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
            CHECK_HIP(launch_vox_cams(ch, hc, stream));
        }
        A.hcams = hc;
    } else if (mode == MODE_VOXEL) {
        // the tallies L_c(k), turned into j_c(k) (images) at the end
        A.Lc = S.take<double>(n_vox * lc_pitch);
        A.lc_pitch = lc_pitch;
        CHECK_HIP(launch_fill_f64(A.Lc, n_vox * lc_pitch, stream));
    } else if (mode == MODE_MIXGRAD) {
        // gradient of a mixture: added to grad
        double* gw = S.take<double>(n_pix);
        CHECK_HIP(launch_grad_weights(gw, dl, ncams, n_cams, n_pix, base_norm, stream));
        A.gw = gw;
        A.grad = grad;
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
        grid_blocks = (int)(need_blocks < full ? need_blocks : full);
    }
    if (keep_rays) {
        // one slice of rw records per wavefront; slots are 32-bit indices
        // (at most three eighths of the available memory; after a kept render
        // on this device, 1.25 times its busiest wavefront's rays per photon)
        const int nw = grid_blocks * (BLOCK / 64);
        size_t avail = 0;
        CHECK_HIP(available_bytes(&avail));
        uint64_t cap = prm->tape_limit > 0 ? (uint64_t)prm->tape_limit
                                           : (uint64_t)(avail / 8 * 3) / sizeof(TapeRec<Real>);
        // (the hint only for the workload it was measured on: another grid or
        // camera set can have many more rays per photon)
        double rate = 0.0;
        tape_key = workload_key(grid, n_cams, cams, prm);
        {
            std::lock_guard<std::mutex> lock(g_mu);
            rate = dev < MAX_DEVICES && g_tape_key[dev] == tape_key ? g_tape_rate[dev] : 0.0;
        }
        if (rate > 0.0 && prm->tape_limit == 0)
            cap = std::min<uint64_t>(cap, (uint64_t)(1.25 * rate * (double)prm->n_photons) + 64 * (uint64_t)nw);
        const uint64_t rw = std::min<uint64_t>(cap / nw, 0xffffffffull / nw);
        kt = new mc_tape();
        kt->magic = 0;
        kt->device = dev;
        kt->nw = nw;
        kt->rw = (uint32_t)rw;
        kt->rec_bytes = sizeof(TapeRec<Real>);
        if (rw < 64 ||
            buf_acquire(BUF_TAPE, sizeof(TapeRec<Real>) * rw * nw, stream, &kt->rec) != hipSuccess ||
            lib_alloc((void**)&kt->wave_count, sizeof(uint32_t) * (nw + 1), stream) != hipSuccess) {
            // no room for the rays: a plain render
            (void)hipGetLastError();
            tape_release(kt, stream);
            kt = nullptr;
            keep_rays = false;
            launch_mode = mode;
        } else {
            A.tp.rec = reinterpret_cast<TapeRec<Real>*>(kt->rec);
            A.tp.rw = kt->rw;
            A.tp.wave_count = kt->wave_count;
            A.tp.overflow = kt->wave_count + nw;
            CHECK_HIP(launch_fill_u32(kt->wave_count, nw + 1, stream));
        }
    }
    if (mode == MODE_MIXGRAD) {
        if (prm->n_photons > 0 && grid_blocks > 0) {
            std::memset(host_counters, 0, sizeof(host_counters));
            const bool tape_occ = mix_tape;  // per_cu was taken for the tape replay
            bool direct = !mix_tape;
            MixPath mp{};
            if (mix_tape && A.mix_full) {
                // the path scores read the sums of 15 collisions per photon
                // (and of the rest), in chunks of at most 4M photons or an
                // eighth of the free memory
                int per_mix = 0;
                size_t avail = 0;
                mp.cap = 15;
                const uint64_t row = sizeof(double) * (mp.cap + 1);
                CHECK_HIP(available_bytes(&avail));
                mp.max_chunk = std::min<uint64_t>(std::min<uint64_t>(prm->n_photons, (uint64_t)1 << 22),
                                                  avail / 8 / row);
                CHECK_HIP(transport_occupancy<Real>(A, MODE_MIXGRAD, tally, &per_mix));
                mp.grid = (int)std::min<uint64_t>((mp.max_chunk + BLOCK - 1) / BLOCK,
                                                  (uint64_t)n_cu * (per_mix > 0 ? per_mix : 1));
                if (mp.max_chunk == 0 || lib_alloc((void**)&mix_rows, row * mp.max_chunk, stream) != hipSuccess) {
                    (void)hipGetLastError();
                    mix_rows = nullptr;
                    mix_tape = false;
                    direct = true;
                } else {
                    mp.rows = mix_rows;
                }
            }
            if (mix_tape) {
                // every estimate's connection term is a ray record of the
                // replay (weight sig * gw * C), binned by tile
                rc = run_tape<Real>(A, TALLY_F64, prm->n_photons, prm->photon_offset, prm->tape_limit,
                                    (int)((int64_t)n_cu * (per_cu > 0 ? per_cu : 1)), n_cu, counters, host_counters,
                                    stats ? &t_transport : nullptr, &t_tape, stream,
                                    workload_key(grid, n_cams, cams, prm) ^ 0x6d6978ull, A.mix_full ? &mp : nullptr);
                if (rc == TAPE_FALLBACK) {
                    // too little room for the records: one photon per lane,
                    // device atomics
                    rc = MC_OK;
                    direct = true;
                    A.tape = 0;
                    std::memset(host_counters, 0, sizeof(host_counters));
                } else if (rc != MC_OK) {
                    goto done;
                } else {
                    tape_counts = true;
                }
            }
            if (direct) {
                // one photon per lane (records, when they fit, binned by tile)
                if (tape_occ) {
                    CHECK_HIP(transport_occupancy<Real>(A, MODE_MIXGRAD, tally, &per_cu));
                    const int64_t full = (int64_t)n_cu * (per_cu > 0 ? per_cu : 1);
                    grid_blocks = (int)(need_blocks < full ? need_blocks : full);
                }
                rc = run_mixgrad<Real>(A, prm, grid_blocks, n_cu, &t_tape, stream);
                if (rc != MC_OK) goto done;
            }
        }
    } else if (A.tape && prm->n_photons > 0 && src) {
        // the rays of the render: no replay
        std::memcpy(host_counters, src->counters, sizeof(host_counters));
        rc = run_tape_kept<Real>(A, tally, src, prm->tape_limit, n_cu, &t_tape, stream);
        if (rc != MC_OK) goto done;
        tape_counts = true;
    } else if (A.tape && prm->n_photons > 0) {
        std::memset(host_counters, 0, sizeof(host_counters));
        rc = run_tape<Real>(A, tally, prm->n_photons, prm->photon_offset, prm->tape_limit,
                            (int)((int64_t)n_cu * (per_cu > 0 ? per_cu : 1)), n_cu, counters, host_counters,
                            stats ? &t_transport : nullptr, &t_tape, stream, workload_key(grid, n_cams, cams, prm));
        if (rc == TAPE_FALLBACK) {
            // tape too small even for one block: device atomics
            rc = MC_OK;
            A.tape = 0;
            CHECK_HIP(transport_occupancy<Real>(A, mode, tally, &per_cu));
            const int64_t full = (int64_t)n_cu * (per_cu > 0 ? per_cu : 1);
            grid_blocks = (int)(need_blocks < full ? need_blocks : full);
            if (stats) {
                CHECK_HIP(hipEventCreate(&ev0));
                CHECK_HIP(hipEventCreate(&ev1));
                CHECK_HIP(hipEventRecord(ev0, stream));
            }
            CHECK_HIP(launch_transport<Real>(A, mode, tally, grid_blocks, stream));
            if (stats) CHECK_HIP(hipEventRecord(ev1, stream));
        } else if (rc != MC_OK) {
            goto done;
        } else {
            tape_counts = true;
        }
    } else if (grid_blocks > 0 && (mode == MODE_TRACE || n_work > 0)) {
        if (stats && !fixed_scratch) {
            CHECK_HIP(hipEventCreate(&ev0));
            CHECK_HIP(hipEventCreate(&ev1));
            CHECK_HIP(hipEventRecord(ev0, stream));
        }
        if constexpr (sizeof(Real) == 4) {
            if (cap) {
                // the gather capture: at most max_waves wavefronts
                grid_blocks = std::min<int>(grid_blocks, (int)(cap->max_waves / (BLOCK / 64)));
                cap->n_waves = (uint32_t)grid_blocks * (BLOCK / 64);
                A.capture = cap->idx;
                A.capture_steps = cap->steps;
                A.cap_first = cap->first;
                A.cap_steps = cap->n_steps;
                // (the capture kernel walks through the buffer only)
                if (grid_blocks < 1 || !A.walk_buf) {
                    rc = MC_ERR_INVALID_ARG;
                    goto done;
                }
                CHECK_HIP(launch_capture(A, grid_blocks, stream));
            }
        }
        if (!cap) CHECK_HIP(launch_transport<Real>(A, launch_mode, tally, grid_blocks, stream));
        if (ev1) CHECK_HIP(hipEventRecord(ev1, stream));
    }

    if (mode == MODE_VOXEL)
        CHECK_HIP(launch_voxel_finish<Real>(images, A.Lc, lc_pitch, betap, n_cams, n_vox, base_norm, stream));
    if (mode == MODE_RENDER) {
        if (k32) CHECK_HIP(launch_kahan_reduce(images, A.img32, n_pix, stream));
        CHECK_HIP(launch_normalize(images, ncams, n_cams, n_pix, base_norm, 1, stream));
        if (images_m2) CHECK_HIP(launch_normalize(images_m2, ncams, n_cams, n_pix, base_norm, 2, stream));
    } else if (mode == MODE_GRAD && k32) {
        CHECK_HIP(launch_kahan_reduce(grad, A.grad32, n_vox, stream));
    }

    if (keep_rays) {
        // the tape is kept only when no slice overflowed
        std::vector<uint32_t> h_wave((size_t)kt->nw + 1);
        CHECK_HIP(hipMemcpyAsync(h_wave.data(), kt->wave_count, sizeof(uint32_t) * (kt->nw + 1),
                                 hipMemcpyDeviceToHost, stream));
        CHECK_HIP(hipMemcpyAsync(kt->counters, counters, sizeof(kt->counters), hipMemcpyDeviceToHost, stream));
        CHECK_HIP(hipStreamSynchronize(stream));
        const bool over = h_wave[kt->nw] != 0;
        {
            uint32_t busiest = 0;
            for (int w = 0; w < kt->nw; ++w) busiest = std::max(busiest, h_wave[w]);
            const double r = (double)busiest * kt->nw / (double)prm->n_photons;
            std::lock_guard<std::mutex> lock(g_mu);
            if (dev < MAX_DEVICES) {
                const double prev = g_tape_key[dev] == tape_key ? g_tape_rate[dev] : 0.0;
                g_tape_rate[dev] = over ? std::max(2.0 * prev, r) : r;
                g_tape_key[dev] = tape_key;
            }
        }
        if (over) {
            tape_release(kt, stream);
        } else {
            kt->magic = TAPE_MAGIC;
            kt->device = dev;
            kt->grid = *grid;
            kt->params = *prm;
            kt->n_cams = n_cams;
            kt->cam_hash = camera_hash(n_cams, cams);
            *keep = kt;
        }
        kt = nullptr;
    }

    if (stats || mode == MODE_TRACE) {
        if (!tape_counts) {
            CHECK_HIP(hipMemcpyAsync(host_counters, counters, sizeof(host_counters), hipMemcpyDeviceToHost, stream));
        }
        CHECK_HIP(hipStreamSynchronize(stream));
        if (stats) {
            stats->photons = mode == MODE_TRACE ? trace_count : n_work;
            stats->events = host_counters[1 + ST_EVENTS];
            stats->le_jobs = host_counters[1 + ST_LE];
            stats->vox_free = host_counters[1 + ST_VFREE];
            stats->vox_conn = host_counters[1 + ST_VCONN];
            stats->esc_top = host_counters[1 + ST_TOP];
            stats->esc_bottom = host_counters[1 + ST_BOTTOM];
            stats->esc_side = host_counters[1 + ST_SIDE];
            stats->rr_killed = host_counters[1 + ST_RR];
            stats->capped = host_counters[1 + ST_CAP];
            if (ev0) {
                float ms = 0.f;
                CHECK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
                t_transport = ms;
            }
            stats->transport_ms = t_transport;
            stats->tape_ms = t_tape;
        }
    }

done:
    if (kt) tape_release(kt, stream);  // an error before the tape was handed over
    if (mix_rows) {
        hipError_t e = hipFreeAsync(mix_rows, stream);
        if (rc == MC_OK && e != hipSuccess) rc = map_err(e);
    }
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (S.base && !fixed_scratch) {
        hipError_t e = hipFreeAsync(S.base, stream);
        if (rc == MC_OK && e != hipSuccess) rc = map_err(e);
    }
    return rc;
}

// Voxelised model, deterministic part: transmittances, then the images
// (images != nullptr) or the gradient (dl, grad).
int run_voxel(const mc_grid* grid, const double* beta, int n_cams, const mc_camera* cams, int n_side,
              const double* j, double* images, const double* dl, double* grad, hipStream_t stream,
              const double* q = nullptr, double* counts = nullptr) {
    int rc = MC_OK;
    const int64_t n_vox = (int64_t)grid->nx * grid->ny * grid->nz;
    const int64_t n_cv = (int64_t)n_cams * n_vox;
    Scratch S;
    VoxArgs A;
    std::memset(&A, 0, sizeof(A));
    size_t bytes = round256(sizeof(HostCam) * n_cams) + round256(sizeof(double) * n_cv) + 256;
    if (grad) bytes += round256(sizeof(double) * n_cv);
    CHECK_HIP(lib_alloc((void**)&S.base, bytes, stream));
    {
        HostCam* dcams = S.take<HostCam>(n_cams);
        int64_t off = 0;
        for (int first = 0; first < n_cams; first += CAM_CHUNK) {
            CamChunk ch;
            std::memset(&ch, 0, sizeof(ch));
            ch.first = first;
            ch.n = n_cams - first < CAM_CHUNK ? n_cams - first : CAM_CHUNK;
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
            CHECK_HIP(launch_vox_cams(ch, dcams, stream));
        }
        A.cams = dcams;
        A.n_pix = off;
    }
    A.nx = grid->nx;
    A.ny = grid->ny;
    A.nz = grid->nz;
    A.dx = grid->dx;
    A.dy = grid->dy;
    A.dz = grid->dz;
    A.n_vox = n_vox;
    A.beta = beta;
    A.n_cams = n_cams;
    A.n_side = n_side;
    A.T = S.take<double>(n_cv);
    A.j = j;
    A.q = q;
    if (counts) {
        // ray counts only (the conditioning)
        CHECK_HIP(launch_fill_f64(counts, n_cv, stream));
        CHECK_HIP(launch_vox_ray_counts(A, counts, stream));
        goto done;
    }
    CHECK_HIP(launch_vox_transmittance(A, stream));
    if (images) {
        A.images = images;
        CHECK_HIP(launch_vox_project(A, stream));
    }
    if (grad) {
        A.dl = dl;
        A.B = S.take<double>(n_cv);
        A.grad = grad;
        CHECK_HIP(launch_fill_f64(A.B, n_cv, stream));
        CHECK_HIP(launch_fill_f64(grad, n_vox, stream));
        CHECK_HIP(launch_vox_backproject(A, stream));
        CHECK_HIP(launch_vox_los_adjoint(A, stream));
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
        case MC_ERR_SCRATCH_LIMIT: return "the call needs more scratch than the fixed 64 MiB of mc_render_noalloc";
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
    if (params->transport != MC_FP32)
        return run<double>(MODE_RENDER, grid, beta, n_cams, cams, params, images, images_m2, nullptr, nullptr, stats,
                           0, 0, 0, nullptr, nullptr, nullptr, s);
    return run<float>(MODE_RENDER, grid, beta, n_cams, cams, params, images, images_m2, nullptr, nullptr, stats, 0,
                      0, 0, nullptr, nullptr, nullptr, s);
}

int mc_render_noalloc(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
                      const mc_params* params, double* images, mc_stats* stats, void* hip_stream) {
    int rc = validate(grid, beta, n_cams, cams, params);
    if (rc != MC_OK) return rc;
    if (!images) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(images)) return MC_ERR_INVALID_ARG;
    void* fixed = nullptr;
    if ((rc = map_err(noalloc_scratch(&fixed))) != MC_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (params->transport != MC_FP32)
        return run<double>(MODE_RENDER, grid, beta, n_cams, cams, params, images, nullptr, nullptr, nullptr, stats,
                           0, 0, 0, nullptr, nullptr, nullptr, s, nullptr, nullptr, 0, nullptr, nullptr, fixed);
    return run<float>(MODE_RENDER, grid, beta, n_cams, cams, params, images, nullptr, nullptr, nullptr, stats, 0,
                      0, 0, nullptr, nullptr, nullptr, s, nullptr, nullptr, 0, nullptr, nullptr, fixed);
}

int mc_capture_gathers(const mc_grid* grid, const float* beta, int n_cams, const mc_camera* cams,
                       const mc_params* params, double* images, uint32_t first_step, uint32_t n_steps,
                       uint32_t max_waves, uint32_t* indices, uint32_t* wave_steps, uint32_t* n_waves,
                       mc_stats* stats, void* hip_stream) {
    int rc = validate(grid, beta, n_cams, cams, params);
    if (rc != MC_OK) return rc;
    if (params->transport != MC_FP32 || params->tally != MC_TALLY_F64) return MC_ERR_INVALID_ARG;
    if (!images || !indices || !wave_steps || !n_waves || n_steps < 1 || max_waves < (uint32_t)(BLOCK / 64))
        return MC_ERR_INVALID_ARG;
    // the capture kernel walks through the buffer: not for grids that take plain loads
    if ((int64_t)grid->nx * grid->ny * grid->nz * (int64_t)sizeof(float) >= ((int64_t)1 << 31) || plain_walk_loads())
        return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(images) || !is_device_ptr(indices) || !is_device_ptr(wave_steps))
        return MC_ERR_INVALID_ARG;
    CaptureArgs cap{indices, wave_steps, first_step, n_steps, max_waves, 0u};
    rc = run<float>(MODE_RENDER, grid, beta, n_cams, cams, params, images, nullptr, nullptr, nullptr, stats, 0, 0, 0,
                    nullptr, nullptr, nullptr, static_cast<hipStream_t>(hip_stream), nullptr, nullptr, 0, nullptr,
                    nullptr, nullptr, &cap);
    *n_waves = cap.n_waves;
    return rc;
}

int mc_grad_beta(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams, const mc_params* params,
                 const double* dl_dimages, double* grad_beta, mc_stats* stats, void* hip_stream) {
    int rc = validate(grid, beta, n_cams, cams, params);
    if (rc != MC_OK) return rc;
    if (!dl_dimages || !grad_beta) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(dl_dimages) || !is_device_ptr(grad_beta)) return MC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (params->transport != MC_FP32)
        return run<double>(MODE_GRAD, grid, beta, n_cams, cams, params, nullptr, nullptr, dl_dimages, grad_beta,
                           stats, 0, 0, 0, nullptr, nullptr, nullptr, s);
    return run<float>(MODE_GRAD, grid, beta, n_cams, cams, params, nullptr, nullptr, dl_dimages, grad_beta, stats,
                      0, 0, 0, nullptr, nullptr, nullptr, s);
}

int mc_render_tape(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
                   const mc_params* params, double* images, mc_stats* stats, void* hip_stream, mc_tape** tape) {
    if (!tape) return MC_ERR_INVALID_ARG;
    *tape = nullptr;
    int rc = validate(grid, beta, n_cams, cams, params);
    if (rc != MC_OK) return rc;
    if (!images) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(images)) return MC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (params->transport != MC_FP32)  // (a mixed-precision render keeps no rays)
        return run<double>(MODE_RENDER, grid, beta, n_cams, cams, params, images, nullptr, nullptr, nullptr, stats,
                           0, 0, 0, nullptr, nullptr, nullptr, s, params->transport == MC_MIXED ? nullptr : tape);
    return run<float>(MODE_RENDER, grid, beta, n_cams, cams, params, images, nullptr, nullptr, nullptr, stats, 0,
                      0, 0, nullptr, nullptr, nullptr, s, tape);
}

int mc_grad_beta_tape(const mc_tape* tape, const mc_grid* grid, const void* beta, int n_cams,
                      const mc_camera* cams, const mc_params* params, const double* dl_dimages, double* grad_beta,
                      mc_stats* stats, void* hip_stream) {
    int rc = validate(grid, beta, n_cams, cams, params);
    if (params->transport == MC_MIXED) return MC_ERR_INVALID_ARG;
    if (rc != MC_OK) return rc;
    if (!tape || tape->magic != TAPE_MAGIC || !dl_dimages || !grad_beta) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != tape->device) return MC_ERR_INVALID_ARG;
    // the same render: grid, cameras and every parameter that shapes the photons
    const mc_grid& g = tape->grid;
    const mc_params& p = tape->params;
    if (g.nx != grid->nx || g.ny != grid->ny || g.nz != grid->nz || g.dx != grid->dx || g.dy != grid->dy ||
        g.dz != grid->dz || tape->n_cams != n_cams || tape->cam_hash != camera_hash(n_cams, cams) ||
        p.albedo != params->albedo || p.g != params->g || p.sun_zenith != params->sun_zenith ||
        p.sun_azimuth != params->sun_azimuth || p.rr_weight != params->rr_weight ||
        p.n_photons != params->n_photons || p.seed != params->seed ||
        p.photon_offset != params->photon_offset || p.n_photons_norm != params->n_photons_norm ||
        p.max_events != params->max_events || p.transport != params->transport)
        return MC_ERR_INVALID_ARG;
    if (!is_device_ptr(beta) || !is_device_ptr(dl_dimages) || !is_device_ptr(grad_beta)) return MC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (params->transport == MC_FP64)
        return run<double>(MODE_GRAD, grid, beta, n_cams, cams, params, nullptr, nullptr, dl_dimages, grad_beta,
                           stats, 0, 0, 0, nullptr, nullptr, nullptr, s, nullptr, tape);
    return run<float>(MODE_GRAD, grid, beta, n_cams, cams, params, nullptr, nullptr, dl_dimages, grad_beta, stats,
                      0, 0, 0, nullptr, nullptr, nullptr, s, nullptr, tape);
}

int mc_voxel_scatter(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams,
                     const mc_params* params, double* j, mc_stats* stats, void* hip_stream) {
    int rc = validate(grid, beta, n_cams, cams, params);
    if (params->transport == MC_MIXED) return MC_ERR_INVALID_ARG;
    if (rc != MC_OK) return rc;
    if (!j || params->tally != MC_TALLY_F64) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(j)) return MC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (params->transport == MC_FP64)
        return run<double>(MODE_VOXEL, grid, beta, n_cams, cams, params, j, nullptr, nullptr, nullptr, stats, 0, 0,
                           0, nullptr, nullptr, nullptr, s);
    return run<float>(MODE_VOXEL, grid, beta, n_cams, cams, params, j, nullptr, nullptr, nullptr, stats, 0, 0, 0,
                      nullptr, nullptr, nullptr, s);
}

int mc_bmc_render(const mc_grid* grid, const void* beta, int n_cams, const mc_camera* cams, const mc_params* params,
                  uint32_t n_per_pixel, double* images, double* images_m2, mc_stats* stats, void* hip_stream) {
    int rc = validate(grid, beta, n_cams, cams, params);
    if (params->transport == MC_MIXED) return MC_ERR_INVALID_ARG;
    if (rc != MC_OK) return rc;
    if (!images || n_per_pixel < 1 || params->tally != MC_TALLY_F64) return MC_ERR_INVALID_ARG;
    if ((uint64_t)pixel_count(n_cams, cams) * n_per_pixel >= ((uint64_t)1 << 62)) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(images) || (images_m2 && !is_device_ptr(images_m2)))
        return MC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (params->transport == MC_FP64)
        return run<double>(MODE_BMC, grid, beta, n_cams, cams, params, images, images_m2, nullptr, nullptr, stats, 0,
                           0, 0, nullptr, nullptr, nullptr, s, nullptr, nullptr, n_per_pixel);
    return run<float>(MODE_BMC, grid, beta, n_cams, cams, params, images, images_m2, nullptr, nullptr, stats, 0, 0,
                      0, nullptr, nullptr, nullptr, s, nullptr, nullptr, n_per_pixel);
}

int mc_render_frozen(const mc_grid* grid, const void* beta_sample, const void* beta_eval, int n_cams,
                     const mc_camera* cams, const mc_params* params, double* images, mc_stats* stats,
                     void* hip_stream) {
    int rc = validate(grid, beta_sample, n_cams, cams, params);
    if (params->transport == MC_MIXED) return MC_ERR_INVALID_ARG;
    if (rc != MC_OK) return rc;
    if (!beta_eval || !images) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta_sample) || !is_device_ptr(beta_eval) || !is_device_ptr(images)) return MC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (params->transport == MC_FP64)
        return run<double>(MODE_RENDER, grid, beta_sample, n_cams, cams, params, images, nullptr, nullptr, nullptr,
                           stats, 0, 0, 0, nullptr, nullptr, nullptr, s, nullptr, nullptr, 0, nullptr, beta_eval);
    return run<float>(MODE_RENDER, grid, beta_sample, n_cams, cams, params, images, nullptr, nullptr, nullptr, stats,
                      0, 0, 0, nullptr, nullptr, nullptr, s, nullptr, nullptr, 0, nullptr, beta_eval);
}

int mc_render_mixture(const mc_grid* grid, const double* beta_air, const double* beta_aer, double sigma,
                      int n_cams, const mc_camera* cams, const mc_params* params, double* images, double* images_m2,
                      mc_stats* stats, void* hip_stream) {
    int rc = validate(grid, beta_air, n_cams, cams, params);
    if (params->transport == MC_MIXED) return MC_ERR_INVALID_ARG;
    if (rc != MC_OK) return rc;
    if (!beta_aer || !images || !(sigma > 0.0) || !std::isfinite(sigma)) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta_air) || !is_device_ptr(beta_aer) || !is_device_ptr(images)) return MC_ERR_INVALID_ARG;
    if (images_m2 && !is_device_ptr(images_m2)) return MC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const MixIn mix{beta_air, beta_aer, sigma, 0};
    if (params->transport == MC_FP64)
        return run<double>(MODE_RENDER, grid, beta_air, n_cams, cams, params, images, images_m2, nullptr, nullptr,
                           stats, 0, 0, 0, nullptr, nullptr, nullptr, s, nullptr, nullptr, 0, &mix);
    return run<float>(MODE_RENDER, grid, beta_air, n_cams, cams, params, images, images_m2, nullptr, nullptr, stats,
                      0, 0, 0, nullptr, nullptr, nullptr, s, nullptr, nullptr, 0, &mix);
}

int mc_grad_mixture(const mc_grid* grid, const double* beta_air, const double* beta_aer, double sigma, int n_cams,
                    const mc_camera* cams, const mc_params* params, const double* dl_dimages, int full,
                    double* grad_beta_aer, mc_stats* stats, void* hip_stream) {
    int rc = validate(grid, beta_air, n_cams, cams, params);
    if (params->transport == MC_MIXED) return MC_ERR_INVALID_ARG;
    if (rc != MC_OK) return rc;
    if (!beta_aer || !dl_dimages || !grad_beta_aer || !(sigma > 0.0) || !std::isfinite(sigma) ||
        (full != 0 && full != 1))
        return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta_air) || !is_device_ptr(beta_aer) || !is_device_ptr(dl_dimages) ||
        !is_device_ptr(grad_beta_aer))
        return MC_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const MixIn mix{beta_air, beta_aer, sigma, full};
    if (params->transport == MC_FP64)
        return run<double>(MODE_MIXGRAD, grid, beta_air, n_cams, cams, params, nullptr, nullptr, dl_dimages,
                           grad_beta_aer, stats, 0, 0, 0, nullptr, nullptr, nullptr, s, nullptr, nullptr, 0, &mix);
    return run<float>(MODE_MIXGRAD, grid, beta_air, n_cams, cams, params, nullptr, nullptr, dl_dimages,
                      grad_beta_aer, stats, 0, 0, 0, nullptr, nullptr, nullptr, s, nullptr, nullptr, 0, &mix);
}

int mc_voxel_render(const mc_grid* grid, const double* beta, int n_cams, const mc_camera* cams, int rays_per_side,
                    const double* j, double* images, void* hip_stream) {
    int rc = validate_scene(grid, beta, n_cams, cams);
    if (rc != MC_OK) return rc;
    if (!j || !images || rays_per_side < 1 || rays_per_side > 64) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(j) || !is_device_ptr(images)) return MC_ERR_INVALID_ARG;
    return run_voxel(grid, beta, n_cams, cams, rays_per_side, j, images, nullptr, nullptr,
                     static_cast<hipStream_t>(hip_stream));
}

int mc_voxel_grad(const mc_grid* grid, const double* beta, int n_cams, const mc_camera* cams, int rays_per_side,
                  const double* j, const double* dl_dimages, const double* cam_weights, double* grad_beta,
                  void* hip_stream) {
    int rc = validate_scene(grid, beta, n_cams, cams);
    if (rc != MC_OK) return rc;
    if (!j || !dl_dimages || !grad_beta || rays_per_side < 1 || rays_per_side > 64) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(j) || !is_device_ptr(dl_dimages) || !is_device_ptr(grad_beta))
        return MC_ERR_INVALID_ARG;
    if (cam_weights && !is_device_ptr(cam_weights)) return MC_ERR_INVALID_ARG;
    return run_voxel(grid, beta, n_cams, cams, rays_per_side, j, nullptr, dl_dimages, grad_beta,
                     static_cast<hipStream_t>(hip_stream), cam_weights);
}

int mc_voxel_conditioning(const mc_grid* grid, int n_cams, const mc_camera* cams, int rays_per_side, double* counts,
                          double* q, void* hip_stream) {
    double one = 1.0;
    int rc = validate_scene(grid, &one, n_cams, cams);
    if (rc != MC_OK) return rc;
    if ((!counts && !q) || rays_per_side < 1 || rays_per_side > 64) return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if ((counts && !is_device_ptr(counts)) || (q && !is_device_ptr(q))) return MC_ERR_INVALID_ARG;
    const int64_t n = (int64_t)n_cams * grid->nx * grid->ny * grid->nz;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    double* c = counts ? counts : q;
    rc = run_voxel(grid, nullptr, n_cams, cams, rays_per_side, nullptr, nullptr, nullptr, nullptr, s, nullptr, c);
    if (rc != MC_OK) return rc;
    if (q) {
        if (counts) {
            hipError_t e = hipMemcpyAsync(q, counts, sizeof(double) * n, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return map_err(e);
        }
        return map_err(launch_vox_invert(q, n, s));
    }
    return MC_OK;
}

int mc_regularizer(const mc_grid* grid, const double* beta, const double* w_layer, double eta, double* grad_beta,
                   double* value, void* hip_stream) {
    if (!grid || !beta || grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return MC_ERR_INVALID_ARG;
    if ((int64_t)grid->nx * grid->ny * grid->nz >= (int64_t)1 << 31) return MC_ERR_INVALID_ARG;
    int rc = precheck_device();
    if (rc != MC_OK) return rc;
    if (!is_device_ptr(beta) || (w_layer && !is_device_ptr(w_layer)) || (grad_beta && !is_device_ptr(grad_beta)) ||
        (value && !is_device_ptr(value)))
        return MC_ERR_INVALID_ARG;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int64_t n = (int64_t)grid->nx * grid->ny * grid->nz;
    double* r = nullptr;
    CHECK_HIP(lib_alloc((void**)&r, sizeof(double) * n, stream));
    if (value) CHECK_HIP(launch_fill_f64(value, 1, stream));
    CHECK_HIP(launch_reg(grid->nx, grid->ny, grid->nz, beta, w_layer, eta, r, grad_beta, value, stream));
done:
    if (r) {
        hipError_t e = hipFreeAsync(r, stream);
        if (rc == MC_OK && e != hipSuccess) rc = map_err(e);
    }
    return rc;
}

int mc_image_residual(int64_t n_pix, const double* images, const double* measured, const double* mask,
                      double* dl_dimages, double* loss, void* hip_stream) {
    if (n_pix < 0 || !images || !measured || !dl_dimages) return MC_ERR_INVALID_ARG;
    int rc = precheck_device();
    if (rc != MC_OK) return rc;
    if (!is_device_ptr(images) || !is_device_ptr(measured) || !is_device_ptr(dl_dimages) ||
        (mask && !is_device_ptr(mask)) || (loss && !is_device_ptr(loss)))
        return MC_ERR_INVALID_ARG;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    if (loss) CHECK_HIP(launch_fill_f64(loss, 1, stream));
    CHECK_HIP(launch_image_residual(n_pix, images, measured, mask, dl_dimages, loss, stream));
done:
    return rc;
}

int mc_gd_step(int64_t n, double* beta, const double* grad, double delta, void* hip_stream) {
    if (n < 0 || !beta || !grad || !std::isfinite(delta)) return MC_ERR_INVALID_ARG;
    int rc = precheck_device();
    if (rc != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(grad)) return MC_ERR_INVALID_ARG;
    return map_err(launch_gd_step(n, beta, grad, delta, static_cast<hipStream_t>(hip_stream)));
}

int mc_camera_noise(int64_t n_pix, const double* images, const double* mask, const double* normals, double* out,
                    double* scale, void* hip_stream) {
    if (n_pix < 0 || !images || !normals || !out) return MC_ERR_INVALID_ARG;
    int rc = precheck_device();
    if (rc != MC_OK) return rc;
    if (!is_device_ptr(images) || !is_device_ptr(normals) || !is_device_ptr(out) || (mask && !is_device_ptr(mask)) ||
        (scale && !is_device_ptr(scale)))
        return MC_ERR_INVALID_ARG;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    unsigned long long* mx = nullptr;
    CHECK_HIP(lib_alloc((void**)&mx, sizeof(unsigned long long), stream));
    CHECK_HIP(launch_fill_u64(mx, 1, stream));
    CHECK_HIP(launch_camera_noise(n_pix, images, mask, normals, mx, out, scale, stream));
done:
    if (mx) {
        hipError_t e = hipFreeAsync(mx, stream);
        if (rc == MC_OK && e != hipSuccess) rc = map_err(e);
    }
    return rc;
}

int mc_recovery_error(int64_t n, const double* beta_hat, const double* beta_true, double* out, void* hip_stream) {
    if (n < 1 || !beta_hat || !beta_true || !out) return MC_ERR_INVALID_ARG;
    int rc = precheck_device();
    if (rc != MC_OK) return rc;
    if (!is_device_ptr(beta_hat) || !is_device_ptr(beta_true)) return MC_ERR_INVALID_ARG;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    double* acc = nullptr;
    double h[3] = {0.0, 0.0, 0.0};
    CHECK_HIP(lib_alloc((void**)&acc, sizeof(double) * 3, stream));
    CHECK_HIP(launch_fill_f64(acc, 3, stream));
    CHECK_HIP(launch_recovery_sums(n, beta_hat, beta_true, acc, stream));
    CHECK_HIP(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, stream));
    CHECK_HIP(hipStreamSynchronize(stream));
    out[0] = (h[0] - h[1]) / h[1];
    out[1] = h[2] / h[1];
done:
    if (acc) {
        hipError_t e = hipFreeAsync(acc, stream);
        if (rc == MC_OK && e != hipSuccess) rc = map_err(e);
    }
    return rc;
}

int mc_recover(const mc_grid* grid, double* beta, int n_cams, const mc_camera* cams, const mc_params* params,
               int rays_per_side, const double* measured, const double* mask, const double* w_layer, double eta,
               double delta, int n_gd, int n_outer, int conditioned, double* cost, void* hip_stream) {
    int rc = validate(grid, beta, n_cams, cams, params);
    if (params->transport == MC_MIXED) return MC_ERR_INVALID_ARG;
    if (rc != MC_OK) return rc;
    if (!measured || params->tally != MC_TALLY_F64 || rays_per_side < 1 || rays_per_side > 64 || n_gd < 1 ||
        n_outer < 0 || !std::isfinite(eta) || !std::isfinite(delta) || conditioned < 0 || conditioned > 2)
        return MC_ERR_INVALID_ARG;
    if ((rc = precheck_device()) != MC_OK) return rc;
    if (!is_device_ptr(beta) || !is_device_ptr(measured) || (mask && !is_device_ptr(mask)) ||
        (w_layer && !is_device_ptr(w_layer)))
        return MC_ERR_INVALID_ARG;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const int64_t n_vox = (int64_t)grid->nx * grid->ny * grid->nz;
    const int64_t n_cv = (int64_t)n_cams * n_vox;
    const int64_t n_pix = pixel_count(n_cams, cams);
    const bool fp32 = params->transport == MC_FP32;
    // j, q: [camera][voxel]; img, dl: pixels; g, r: voxels; two scalars
    const size_t bytes = round256(sizeof(double) * n_cv) * (conditioned ? 2 : 1) +
                         round256(sizeof(double) * n_pix) * 2 + round256(sizeof(double) * n_vox) * 2 +
                         round256(sizeof(float) * n_vox) + 256 + 256;
    Scratch S;
    double *j = nullptr, *q = nullptr, *img = nullptr, *dl = nullptr, *g = nullptr, *r = nullptr, *scal = nullptr;
    float* bf = nullptr;
    double h[2] = {0.0, 0.0};
    CHECK_HIP(lib_alloc((void**)&S.base, bytes, stream));
    j = S.take<double>(n_cv);
    if (conditioned) q = S.take<double>(n_cv);
    img = S.take<double>(n_pix);
    dl = S.take<double>(n_pix);
    g = S.take<double>(n_vox);
    r = S.take<double>(n_vox);
    bf = S.take<float>(n_vox);
    scal = S.take<double>(2);
    if (q) {
        rc = run_voxel(grid, nullptr, n_cams, cams, rays_per_side, nullptr, nullptr, nullptr, nullptr, stream,
                       nullptr, q);
        if (rc != MC_OK) goto done;
        if (conditioned == 1) CHECK_HIP(launch_vox_invert(q, n_cv, stream));
    }
    for (int it = 0; it < n_outer; ++it) {
        // j at the current beta, with the photons of seed + it
        mc_params P = *params;
        P.seed = params->seed + (uint64_t)it;
        if (fp32) {
            CHECK_HIP(launch_d2f(n_vox, beta, bf, stream));
            rc = run<float>(MODE_VOXEL, grid, bf, n_cams, cams, &P, j, nullptr, nullptr, nullptr, nullptr, 0, 0, 0,
                            nullptr, nullptr, nullptr, stream);
        } else {
            rc = run<double>(MODE_VOXEL, grid, beta, n_cams, cams, &P, j, nullptr, nullptr, nullptr, nullptr, 0, 0, 0,
                             nullptr, nullptr, nullptr, stream);
        }
        if (rc != MC_OK) goto done;
        for (int d = 0; d < n_gd; ++d) {
            rc = run_voxel(grid, beta, n_cams, cams, rays_per_side, j, img, nullptr, nullptr, stream);
            if (rc != MC_OK) goto done;
            CHECK_HIP(launch_fill_f64(scal, 2, stream));
            CHECK_HIP(launch_image_residual(n_pix, img, measured, mask, dl, scal, stream));
            rc = run_voxel(grid, beta, n_cams, cams, rays_per_side, j, nullptr, dl, g, stream, q);
            if (rc != MC_OK) goto done;
            if (eta != 0.0)
                CHECK_HIP(launch_reg(grid->nx, grid->ny, grid->nz, beta, w_layer, eta, r, g, scal + 1, stream));
            if (cost) {
                CHECK_HIP(hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, stream));
                CHECK_HIP(hipStreamSynchronize(stream));
                cost[(int64_t)it * n_gd + d] = h[0] + eta * h[1];
            }
            CHECK_HIP(launch_gd_step(n_vox, beta, g, delta, stream));
        }
    }
done:
    if (S.base) {
        hipError_t e = hipFreeAsync(S.base, stream);
        if (rc == MC_OK && e != hipSuccess) rc = map_err(e);
    }
    (void)hipStreamSynchronize(stream);  // h was a copy target
    return rc;
}

int mc_release_memory(void) {
    int rc = precheck_device();
    if (rc != MC_OK) return rc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev >= MAX_DEVICES) return MC_ERR_HIP;
    hipMemPool_t pool = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        pool = g_pool[dev];
        for (int i = 0; i < N_BUFS; ++i) {
            CachedBuf& b = g_buf[dev][i];
            if (b.in_use || !b.ptr) continue;
            if (hipFree(b.ptr) != hipSuccess) return MC_ERR_HIP;
            b.ptr = nullptr;
            b.bytes = 0;
        }
    }
    if (!pool) return MC_OK;
    return map_err(hipMemPoolTrimTo(pool, 0));
}

int mc_tape_free(mc_tape* tape, void* hip_stream) {
    if (!tape) return MC_OK;
    if (tape->magic != TAPE_MAGIC) return MC_ERR_INVALID_ARG;
    tape_release(tape, static_cast<hipStream_t>(hip_stream));
    return MC_OK;
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
    if (params->transport != MC_FP32)
        return run<double>(MODE_TRACE, grid, beta, n_cams, cams, params, nullptr, nullptr, nullptr, nullptr,
                           nullptr, first_pid, count, max_rec, events, pix, paths, s);
    return run<float>(MODE_TRACE, grid, beta, n_cams, cams, params, nullptr, nullptr, nullptr, nullptr, nullptr,
                      first_pid, count, max_rec, events, pix, paths, s);
}

}  // extern "C"
