// C ABI of libgaca (include/gaca.h): context, problem (mesh, frequencies, tree,
// partition, device geometry), build (near field + far-field 3D-ACA), export, apply.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <limits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <functional>
#include <numeric>
#include <vector>

#include "host.h"
#include "kernels.h"

using namespace gaca;

// ---------------------------------------------------------------------------------------
// device buffers with accounting against max_device_bytes
struct gaca_context {
    int device = 0;
    int n_cu = 256;           // compute units of the device
    hipStream_t stream = nullptr;
    uint64_t limit = 0;       // 0: none
    std::atomic<uint64_t> in_use{0};   // builds of different problems may run in parallel threads
    // problems made on the context; gaca_context_destroy only marks the context, which is
    // deleted with its last problem (handles may then be destroyed in any order)
    std::atomic<int> refs{0};
    std::atomic<bool> destroy_requested{false};
    // far-field stream sets (four streams each) of destroyed problems, taken again by later
    // problems: the runtime spreads streams over a few hardware queues in creation order, so
    // fresh streams for every problem can land two face classes on one queue, where they
    // run one after the other
    std::mutex stream_mu;
    std::vector<std::array<hipStream_t, 4>> stream_pool;
    ~gaca_context() {
        for (auto &set : stream_pool)
            for (hipStream_t st : set) (void)hipStreamDestroy(st);
    }
};

namespace {

// Host time spent in device-memory management calls (allocation, mapping, release), for
// the verbose progress lines.
static std::atomic<int64_t> g_mem_ns{0}, g_mem_calls{0};
static std::atomic<int> g_mem_verbose{0};   // report memory calls slower than 10 ms
struct MemTimer {
    const char *what;
    size_t size;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    explicit MemTimer(const char *w = "", size_t sz = 0) : what(w), size(sz) {}
    ~MemTimer() {
        const int64_t ns =
            std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0).count();
        g_mem_ns += ns;
        ++g_mem_calls;
        if (g_mem_verbose.load() && ns > 10000000)
            std::fprintf(stderr, "gaca memory: %s of %.1f MiB took %.1f ms\n", what, size / 1048576.0, ns / 1e6);
    }
};

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    gaca_context *ctx = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (ptr) {
            MemTimer mt("hipFree", bytes);
            (void)hipFree(ptr);
            if (ctx) ctx->in_use -= bytes;
        }
        ptr = nullptr;
        bytes = 0;
    }
    void alloc(gaca_context *c, size_t nbytes) {
        release();
        ctx = c;
        if (nbytes == 0) nbytes = 16;
        if (c->limit && c->in_use + nbytes > c->limit)
            throw Error{GACA_ERR_OOM, "device memory cap exceeded (max_device_bytes)"};
        hipError_t e;
        {
            MemTimer mt("hipMalloc", nbytes);
            e = hipMalloc(&ptr, nbytes);
        }
        if (e != hipSuccess) {
            ptr = nullptr;
            (void)hipGetLastError();
            throw Error{GACA_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
        }
        bytes = nbytes;
        c->in_use += nbytes;
    }
    void swap(DevBuf &o) {
        std::swap(ptr, o.ptr);
        std::swap(bytes, o.bytes);
        std::swap(ctx, o.ctx);
    }
    template <class T>
    T *as() const { return reinterpret_cast<T *>(ptr); }
    template <class T>
    void upload(gaca_context *c, const std::vector<T> &v) {
        alloc(c, v.size() * sizeof(T));
        if (!v.empty())
            GACA_HIP_CHECK(hipMemcpy(ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    }
};

// Device buffer that grows in place: a virtual address range is reserved once and physical
// chunks are mapped behind its end as needed (HIP virtual memory), so growing never copies
// and never holds the old and the new buffer at once; shrinking unmaps the tail.  Where the
// virtual-memory calls are not available it falls back to allocate-copy-free.
struct GrowBuf {
    void *ptr = nullptr;      // base address
    size_t bytes = 0;         // usable (mapped) bytes
    gaca_context *ctx = nullptr;
    bool vmm = false;
    size_t reserved = 0, gran = 0;
    int device = 0;
    std::vector<std::pair<hipMemGenericAllocationHandle_t, size_t>> chunks;
    DevBuf plain;             // fallback storage
    std::string last_fail;    // the call that failed last (for error messages)
    GrowBuf() = default;
    GrowBuf(const GrowBuf &) = delete;
    GrowBuf &operator=(const GrowBuf &) = delete;
    ~GrowBuf() { release(); }
    template <class T>
    T *as() const { return reinterpret_cast<T *>(ptr); }
    void swap(GrowBuf &o) {
        std::swap(ptr, o.ptr);
        std::swap(bytes, o.bytes);
        std::swap(ctx, o.ctx);
        std::swap(vmm, o.vmm);
        std::swap(reserved, o.reserved);
        std::swap(gran, o.gran);
        std::swap(device, o.device);
        chunks.swap(o.chunks);
        plain.swap(o.plain);
        last_fail.swap(o.last_fail);
    }

    void release() {
        if (vmm && ptr) {
            MemTimer mt("release of a mapped buffer", bytes);
            (void)hipDeviceSynchronize();
            size_t off = 0;
            for (auto &c : chunks) {
                (void)hipMemUnmap(static_cast<char *>(ptr) + off, c.second);
                (void)hipMemRelease(c.first);
                if (ctx) ctx->in_use -= c.second;
                off += c.second;
            }
            chunks.clear();
            (void)hipMemAddressFree(ptr, reserved);
        }
        plain.release();
        ptr = nullptr;
        bytes = 0;
        reserved = 0;
        vmm = false;
    }

    // map at least `add` more bytes as chunks of one size, `gran`, fixed at the first use (the
    // runtime refused access rights on some mixes of chunk sizes; uniform chunks were always
    // accepted); false when out of memory
    bool map_more(size_t add) {
        size_t left = (add + gran - 1) / gran * gran;
        while (left > 0) {
            if (!map_chunk(gran)) return false;
            left -= gran;
        }
        return true;
    }

    bool map_chunk(size_t sz) {
        if (bytes + sz > reserved) return false;
        if (ctx->limit && ctx->in_use + sz > ctx->limit) return false;
        MemTimer mt("mapping a chunk", sz);
        hipMemAllocationProp prop{};
        prop.type = hipMemAllocationTypePinned;
        prop.location.type = hipMemLocationTypeDevice;
        prop.location.id = device;
        hipMemGenericAllocationHandle_t hd{};
        auto fail = [&](const char *what, hipError_t e) {
            last_fail = std::string(what) + " of " + std::to_string(sz >> 20) + " MiB at offset " +
                        std::to_string(bytes >> 20) + " MiB: " + hipGetErrorString(e);
            (void)hipGetLastError();
            return false;
        };
        hipError_t e = hipMemCreate(&hd, sz, &prop, 0);
        if (e != hipSuccess) return fail("hipMemCreate", e);
        char *at = static_cast<char *>(ptr) + bytes;
        e = hipMemMap(at, sz, 0, hd, 0);
        if (e != hipSuccess) {
            (void)hipMemRelease(hd);
            return fail("hipMemMap", e);
        }
        hipMemAccessDesc desc{};
        desc.location.type = hipMemLocationTypeDevice;
        desc.location.id = device;
        desc.flags = hipMemAccessFlagsProtReadWrite;
        e = hipMemSetAccess(at, sz, &desc, 1);
        if (e != hipSuccess) {
            (void)hipMemUnmap(at, sz);
            (void)hipMemRelease(hd);
            return fail("hipMemSetAccess", e);
        }
        chunks.emplace_back(hd, sz);
        bytes += sz;
        ctx->in_use += sz;
        return true;
    }

    // first use: reserve the address range (the device's memory size) and map `need` bytes
    void start(gaca_context *c, size_t need) {
        release();
        ctx = c;
        device = c->device;
        int supported = 0;
        size_t free_b = 0, total_b = 0;
        hipMemAllocationProp prop{};
        prop.type = hipMemAllocationTypePinned;
        prop.location.type = hipMemLocationTypeDevice;
        prop.location.id = device;
        if (hipDeviceGetAttribute(&supported, hipDeviceAttributeVirtualMemoryManagementSupported, device) ==
                hipSuccess &&
            supported && hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
            hipMemGetAllocationGranularity(&gran, &prop, hipMemAllocationGranularityMinimum) == hipSuccess &&
            gran > 0) {
            // uniform chunks of 64 MiB to 1 GiB (a power of two near a sixteenth of the
            // first request; a multiple of the granularity)
            size_t chunk = (size_t)64 << 20;
            while (chunk < ((size_t)1 << 30) && chunk * 16 < need) chunk *= 2;
            gran = (chunk + gran - 1) / gran * gran;
            reserved = (total_b + gran - 1) / gran * gran;
            if (hipMemAddressReserve(&ptr, reserved, 0, nullptr, 0) == hipSuccess) {
                vmm = true;
                if (!map_more(std::max<size_t>(need, gran))) {
                    const std::string why = last_fail;
                    release();
                    throw Error{GACA_ERR_OOM, "device memory exhausted (mapping a growable buffer: " + why + ")"};
                }
                return;
            }
            ptr = nullptr;
        }
        (void)hipGetLastError();
        vmm = false;
        plain.alloc(c, std::max<size_t>(need, 16));
        ptr = plain.ptr;
        bytes = plain.bytes;
    }

    // at least `need` bytes, keeping the first `used`; work on `st` that uses the buffer
    // must be complete or ordered before the copy of the fallback path
    void grow(gaca_context *c, size_t need, size_t used, hipStream_t st) {
        if (!ptr) {
            start(c, need);
            return;
        }
        if (need <= bytes) return;
        if (vmm) {
            // grow by half the size, at most 4 GiB (mapped memory is never over-committed by
            // much), at least 256 MiB; short of that, by what is needed
            const size_t step = std::min<size_t>(bytes / 2, (size_t)4 << 30);
            const size_t target = bytes + std::max(need - bytes, std::max<size_t>(step, (size_t)256 << 20));
            while (bytes < target)
                if (!map_more(gran)) break;
            if (bytes >= need) return;
            // the mapping could not be extended: move to an ordinary allocation
            if (g_mem_verbose.load())
                std::fprintf(stderr, "gaca memory: mapping failed (%s), copying %.1f MiB to a plain allocation\n",
                             last_fail.c_str(), used / 1048576.0);
            DevBuf nb;
            nb.alloc(c, std::max(need, bytes + bytes / 2));
            if (used > 0)
                GACA_HIP_CHECK(hipMemcpyAsync(nb.ptr, ptr, std::min(used, bytes), hipMemcpyDeviceToDevice, st));
            GACA_HIP_CHECK(hipStreamSynchronize(st));
            release();
            ctx = c;
            std::swap(plain.ptr, nb.ptr);
            std::swap(plain.bytes, nb.bytes);
            plain.ctx = c;
            nb.ctx = nullptr;
            ptr = plain.ptr;
            bytes = plain.bytes;
            return;
        }
        DevBuf nb;
        nb.alloc(c, std::max(need, bytes + bytes / 2));
        if (used > 0)
            GACA_HIP_CHECK(hipMemcpyAsync(nb.ptr, plain.ptr, std::min(used, bytes), hipMemcpyDeviceToDevice, st));
        GACA_HIP_CHECK(hipStreamSynchronize(st));
        std::swap(plain.ptr, nb.ptr);
        std::swap(plain.bytes, nb.bytes);
        ptr = plain.ptr;
        bytes = plain.bytes;
    }

    // drop the mapped tail beyond `used` bytes (whole chunks only; used = 0 unmaps all and
    // keeps the address range); the buffer must be idle
    void shrink(size_t used) {
        if (!vmm || chunks.empty()) return;
        if (used > bytes) return;
        MemTimer mt("shrinking a mapped buffer", bytes);
        (void)hipDeviceSynchronize();
        while (!chunks.empty() && bytes - chunks.back().second >= used) {
            const auto c = chunks.back();
            bytes -= c.second;
            (void)hipMemUnmap(static_cast<char *>(ptr) + bytes, c.second);
            (void)hipMemRelease(c.first);
            ctx->in_use -= c.second;
            chunks.pop_back();
        }
    }
};

// Pinned host staging buffer (per-iteration uploads and status read-back).
struct PinnedBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf &) = delete;
    PinnedBuf &operator=(const PinnedBuf &) = delete;
    ~PinnedBuf() {
        if (ptr) (void)hipHostFree(ptr);
    }
    void ensure(size_t need) {
        if (need <= bytes && ptr) return;
        MemTimer mt("pinned host allocation", need);
        if (ptr) (void)hipHostFree(ptr);
        ptr = nullptr;
        const size_t want = std::max<size_t>({need, bytes + bytes / 2, 4096});
        bytes = 0;
        GACA_HIP_CHECK(hipHostMalloc(&ptr, want, 0));
        bytes = want;
    }
    template <class T>
    T *as() const { return reinterpret_cast<T *>(ptr); }
};

// Far-field working memory, kept by the problem across builds (it only grows).
struct FarScratch {
    DevBuf blk, state, coef, hs, fs, usedk, uw, part, act, map_chunk, map_tile, status, copies,
        gathers, rec_ws;
    GrowBuf hpool, fgpool;
    PinnedBuf h_act, h_status, h_copies, h_gathers, h_blk, h_out;
};

template <class F>
gaca_status guarded(F &&fn) {
    try {
        fn();
        return GACA_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return GACA_ERR_OOM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return GACA_ERR_INVALID_ARG;
    }
}

#define REQUIRE(cond, msg) \
    do {                   \
        if (!(cond)) throw Error{GACA_ERR_INVALID_ARG, msg}; \
    } while (0)

}  // namespace

// A problem's reference to its context, declared first among the problem's members so that
// it is released last (the other members account their device memory in the context).
struct CtxRef {
    gaca_context *c = nullptr;
    ~CtxRef() {
        if (c && --c->refs == 0 && c->destroy_requested) delete c;
    }
};

struct gaca_problem {
    CtxRef ctxref;
    gaca_context *ctx = nullptr;
    // operators built on the problem; gaca_problem_destroy only marks the problem, which is
    // deleted with its last operator
    std::atomic<int> nops{0};
    std::atomic<bool> destroy_requested{false};
    void attach(gaca_context *c) {
        ctx = c;
        ctxref.c = c;
        ctx->refs += 1;
    }
    gaca_options opt{};
    std::string autotune_path;    // copy of opt.autotune_cache (opt points at it)
    int tuned_tl = 0, tuned_ts = 0;   // face-ACA workgroup sizes chosen by the autotuner
    int tune_state = 0;               // 0 none, 1 measured by this problem, 2 read from the cache
    // faces per far block that the last build of each operator kind (slot 6: joint builds)
    // stored, the start of the next build's batch estimate (0 = no build yet)
    double faces_per_block[7] = {0, 0, 0, 0, 0, 0, 0};
    gaca_scheme scheme = GACA_COLLOCATION_P0;
    bool synthetic = false;       // dense-tensor problem of gaca_compress_tensor
    HostMesh mesh;
    // P1 scheme: the degrees of freedom are the vertices (points at the vertices, boxes of
    // their patches, for the cluster tree) and each vertex's patch (tree order CSR)
    HostMesh dofs;
    std::vector<int32_t> pptr, ptri, ploc;
    std::vector<double> patch_prefix;    // prefix sums of the patch sizes in tree order
    double p1_near_points = 0.0;         // quadrature points of the near field per frequency
    DevBuf d_p1i;
    ClusterTree tree;
    Partition part;
    int32_t L = 0;
    std::vector<double> s_re, s_im;
    bool mirror = false;
    int64_t M = 0;
    std::vector<int64_t> inv_perm;
    // device geometry / tables
    DevBuf d_geo, d_geo32, d_quad, d_freq, d_perm;
    GeoDev g{};
    QuadDev q{};
    FreqDev f{};
    // near field layout
    std::vector<NearBlockDev> nblocks;
    int64_t near_elems = 0;
    DevBuf d_nblocks;
    DevBuf d_pairs[kNumTiers];
    int64_t npairs[kNumTiers] = {0, 0, 0, 0, 0, 0};
    int kid(gaca_kernel k) const {
        if (scheme == GACA_GALERKIN_P1) return k == GACA_HYP ? 4 : 5;
        return scheme == GACA_GALERKIN_P0 ? 2 : scheme == GACA_COLLOCATION_P1 ? 3 : (int)k;
    }
    bool p1() const { return scheme == GACA_COLLOCATION_P1 || scheme == GACA_GALERKIN_P1; }
    // leaves for the apply
    std::vector<int32_t> leaf_r0, leaf_m;
    // far-field launch classes run concurrently on these streams (default priority)
    hipStream_t far_streams[4] = {nullptr, nullptr, nullptr, nullptr};
    bool far_streams_ready = false;
    FarScratch fsc;
    // mapped factor / fibre arenas of destroyed H-matrices, reused by the next build (mapping
    // fresh pages costs milliseconds per GiB); guarded by spare_mu
    std::mutex spare_mu;
    // leaf CSR of the partition (leaf -> far / near blocks covering its rows), shared by the
    // applies of every operator of the problem
    std::mutex leaf_mu;
    bool leaf_ready = false;
    DevBuf d_leaf_r0, d_leaf_m, d_lfp, d_lfi, d_lnp, d_lni;
    // VALU apply workspace (X, Y in tree order, z, t, y) handed back by destroyed operators
    DevBuf ws_spare[5];
    // near-field storage handed back by destroyed operators (slot kernel & 1)
    DevBuf near_spare[2];
    // far-field result tables of destroyed operators (device: meta, cross meta, cross offsets,
    // fibre offsets, block list; host: the same tables), by slot kernel & 1: taking them back
    // spares the next build the allocation and first touch of tens of MB
    DevBuf tab_spare[2][5];
    std::vector<FarMeta> meta_spare[2];
    std::vector<CrossMeta> cmeta_spare[2];
    std::vector<int64_t> coff_spare[2], foff_spare[2];
    GrowBuf spare_arena[2], spare_fib[2];
    ~gaca_problem();
};

struct gaca_hmatrix {
    gaca_problem *p = nullptr;
    ~gaca_hmatrix();
    std::unique_ptr<gaca_problem> owned_problem;   // synthetic problems
    int kernel = 0;
    gaca_precision prec = GACA_FP64;
    int32_t rcap = 0;
    int64_t nfar = 0;
    double eps_aca_used = 0.0;
    DevBuf d_near, d_meta, d_cmeta, d_cross_off, d_fib_off, d_far4;
    DevBuf d_gcqw;                 // gCQ quadrature weights of the last history step
    // near blocks compressed along the frequencies (option near_aca): the operator's own block
    // table, the faces and fibres of the compressed blocks and the dense arena of the others
    bool near_aca = false;
    DevBuf d_nblk_own;
    GrowBuf n_faces, n_fib, n_dense;
    std::vector<NearBlockDev> nblk_host;
    int64_t near_faces_elems = 0, near_fib_elems = 0, near_dense_elems = 0;
    GrowBuf d_arena, d_fib;   // factor and fibre arenas (grow in place)
    std::vector<FarMeta> meta;
    std::vector<CrossMeta> cmeta;
    std::vector<int64_t> cross_off, fib_off;
    gaca_stats st{};
    std::vector<int64_t> freq_hist;
    // apply workspace
    int32_t ws_nrhs = -1, ws_mode = -1, ws_dtype = -1, ws_cb = 1;
    DevBuf d_xp, d_yp, d_z, d_t, d_toff, d_zoff, d_yb, d_yoff;
    DevBuf d_tn, d_tnoff;   // T of the compressed near blocks (option near_aca, SUM mode)
    hipEvent_t apply_ev[2] = {nullptr, nullptr};   // fork / join of the VALU SUM apply's side stream
    DevBuf d_mz, d_mt, d_mtitems, d_mttile0, d_mtrows, d_mzitems, d_mzoff, d_msumrho;   // matrix-core apply
};

gaca_problem::~gaca_problem() {
    if (far_streams_ready) {
        std::lock_guard<std::mutex> lk(ctx->stream_mu);
        ctx->stream_pool.push_back({far_streams[0], far_streams[1], far_streams[2], far_streams[3]});
    }
}

gaca_hmatrix::~gaca_hmatrix() {
    for (hipEvent_t e : apply_ev)
        if (e) (void)hipEventDestroy(e);
    if (p && !owned_problem && --p->nops == 0 && p->destroy_requested) delete p;
}

// ---------------------------------------------------------------------------------------
extern "C" {

int gaca_abi_version(void) { return GACA_ABI_VERSION; }
const char *gaca_last_error(void) { return last_error(); }
void gaca_options_default(gaca_options *opt) {
    if (opt) options_default(opt);
}

gaca_status gaca_context_create(int device, void *hip_stream, gaca_context **out) {
    return guarded([&] {
        REQUIRE(out, "out is null");
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
            (void)hipGetLastError();
            throw Error{GACA_ERR_STATE, "no HIP device available"};
        }
        REQUIRE(device >= 0 && device < count, "device index out of range");
        GACA_HIP_CHECK(hipSetDevice(device));
        // device address of the allocation-free apply's scratch array on this device
        GACA_HIP_CHECK(scratch_setup(device));
        auto *c = new gaca_context;
        c->device = device;
        c->stream = reinterpret_cast<hipStream_t>(hip_stream);
        int ncu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
            ncu > 0)
            c->n_cu = ncu;
        else
            (void)hipGetLastError();
        *out = c;
    });
}

gaca_status gaca_context_memory(const gaca_context *ctx, uint64_t *in_use) {
    return guarded([&] {
        REQUIRE(ctx && in_use, "null argument");
        *in_use = ctx->in_use.load();
    });
}

gaca_status gaca_context_destroy(gaca_context *ctx) {
    if (!ctx) return GACA_OK;
    ctx->destroy_requested = true;
    if (ctx->refs.load() == 0) delete ctx;
    return GACA_OK;
}

// P1 degrees of freedom: one per vertex.  The cluster tree splits them by vertex position
// and tests admissibility on the boxes of their patches (the supports of the trial
// functions), so that an admissible pair has separated supports.
static void p1_dofs(const HostMesh &m, HostMesh &d) {
    const int64_t nv = m.nv, T = m.M;
    d.nv = nv;
    d.M = nv;
    d.cen = m.xyz;
    d.vmin.assign(3 * nv, std::numeric_limits<double>::infinity());
    d.vmax.assign(3 * nv, -std::numeric_limits<double>::infinity());
    std::vector<int32_t> cnt(nv, 0);
    for (int64_t t = 0; t < T; ++t)
        for (int c = 0; c < 3; ++c) {
            const int32_t v = m.tri[3 * t + c];
            ++cnt[v];
            for (int k = 0; k < 3; ++k) {
                d.vmin[3 * v + k] = std::min(d.vmin[3 * v + k], m.vmin[3 * t + k]);
                d.vmax[3 * v + k] = std::max(d.vmax[3 * v + k], m.vmax[3 * t + k]);
            }
        }
    for (int64_t v = 0; v < nv; ++v)
        if (cnt[v] == 0) throw Error{GACA_ERR_INVALID_ARG, "P1 scheme: a vertex belongs to no triangle"};
}

// Block lists of a partition into caller arrays (row_start, m, col_start, n each).
static void write_blocks(const Partition &part, int64_t capacity, int64_t *far4, int64_t *n_far,
                         int64_t *near4, int64_t *n_near) {
    *n_far = (int64_t)part.far.size();
    *n_near = (int64_t)part.near.size();
    if ((int64_t)part.far.size() > capacity || (int64_t)part.near.size() > capacity)
        throw Error{GACA_ERR_INVALID_ARG, "block list capacity too small"};
    for (size_t b = 0; b < part.far.size(); ++b)
        for (int k = 0; k < 4; ++k) far4[4 * b + k] = part.far[b][k];
    for (size_t b = 0; b < part.near.size(); ++b)
        for (int k = 0; k < 4; ++k) near4[4 * b + k] = part.near[b][k];
}

gaca_status gaca_partition_host(const double *xyz, int64_t nv, const int32_t *tri, int64_t M,
                                int32_t leaf_size, double eta, int64_t *perm,
                                int64_t capacity, int64_t *far4, int64_t *n_far,
                                int64_t *near4, int64_t *n_near) {
    return guarded([&] {
        REQUIRE(perm && n_far && n_near, "null output");
        REQUIRE(eta > 0.0, "eta must be > 0");
        HostMesh mesh;
        mesh.init(xyz, nv, tri, M);
        ClusterTree tree;
        tree.build(mesh, leaf_size);
        Partition part;
        part.build(tree, eta);
        std::copy(tree.perm.begin(), tree.perm.end(), perm);
        write_blocks(part, capacity, far4, n_far, near4, n_near);
    });
}

gaca_status gaca_partition_host_p1(const double *xyz, int64_t nv, const int32_t *tri, int64_t M,
                                   int32_t leaf_size, double eta, int64_t *perm,
                                   int64_t capacity, int64_t *far4, int64_t *n_far,
                                   int64_t *near4, int64_t *n_near) {
    return guarded([&] {
        REQUIRE(perm && n_far && n_near, "null output");
        REQUIRE(eta > 0.0, "eta must be > 0");
        HostMesh mesh, dofs;
        mesh.init(xyz, nv, tri, M);
        p1_dofs(mesh, dofs);
        ClusterTree tree;
        tree.build(dofs, leaf_size);
        Partition part;
        part.build(tree, eta);
        std::copy(tree.perm.begin(), tree.perm.end(), perm);
        write_blocks(part, capacity, far4, n_far, near4, n_near);
    });
}

gaca_status gaca_quadrature_rule(int kind, int n, double *nodes, double *weights) {
    return guarded([&] {
        REQUIRE(nodes && weights, "null output");
        if (kind == 0) {
            REQUIRE(n >= 1 && n <= 128, "n must be in [1, 128]");
            Rule1D r = gauss_legendre01(n);
            for (int i = 0; i < n; ++i) {
                nodes[i] = r.x[i];
                weights[i] = r.w[i];
            }
        } else if (kind == 1) {
            REQUIRE(n == 6, "the triangle rule has 6 points");
            double b[6][3], w[6];
            triangle6(b, w);
            for (int i = 0; i < 6; ++i) {
                for (int k = 0; k < 3; ++k) nodes[3 * i + k] = b[i][k];
                weights[i] = w[i];
            }
        } else {
            throw Error{GACA_ERR_INVALID_ARG, "unknown rule kind"};
        }
    });
}

// Quadrature tables in device memory (every scheme).
static void upload_quad(gaca_problem *p) {
    gaca_context *ctx = p->ctx;
    double bary[6][3], w6[6];
    triangle6(bary, w6);
    Rule1D r4 = gauss_legendre01(p->opt.quad_mid), r8 = gauss_legendre01(p->opt.quad_near),
           rd = gauss_legendre01(p->opt.n_duffy), rg = gauss_legendre01(p->opt.n_galerkin),
           rs = gauss_legendre01(p->opt.n_touch);
    std::vector<double> qt;
    auto push_rule = [&](const Rule1D &r) {
        size_t off = qt.size();
        for (size_t i = 0; i < r.x.size(); ++i) {
            qt.push_back(r.x[i]);
            qt.push_back(r.w[i]);
        }
        return off;
    };
    Rule1D rth = gauss_legendre01(kGalerkinNTheta);
    size_t o4 = push_rule(r4), o8 = push_rule(r8), od = push_rule(rd), og = push_rule(rg),
           oth = push_rule(rth), os = push_rule(rs);
    size_t o6 = qt.size();
    for (int q = 0; q < 6; ++q) {
        qt.push_back(bary[q][0]);
        qt.push_back(bary[q][1]);
        qt.push_back(bary[q][2]);
        qt.push_back(w6[q]);
    }
    p->d_quad.upload(ctx, qt);
    const double *Q = p->d_quad.as<double>();
    p->q.n4 = p->opt.quad_mid;
    p->q.n8 = p->opt.quad_near;
    p->q.nd = p->opt.n_duffy;
    p->q.ng = p->opt.n_galerkin;
    p->q.ns = p->opt.n_touch;
    p->q.gs = Q + os;
    p->q.g4 = Q + o4;
    p->q.g8 = Q + o8;
    p->q.gd = Q + od;
    p->q.gg = Q + og;
    p->q.r6 = Q + o6;
    p->q.nth = kGalerkinNTheta;
    p->q.gth = Q + oth;
}

// Leaves of the cluster tree in tree order (the row groups of the apply).
static void set_leaves(gaca_problem *p) {
    p->leaf_r0.clear();
    p->leaf_m.clear();
    for (const auto &nd : p->tree.nodes)
        if (nd.child[0] < 0) {
            p->leaf_r0.push_back((int32_t)nd.start);
            p->leaf_m.push_back((int32_t)nd.size);
        }
    std::vector<size_t> order(p->leaf_r0.size());
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(),
              [&](size_t a, size_t b) { return p->leaf_r0[a] < p->leaf_r0[b]; });
    std::vector<int32_t> r0s, ms;
    for (size_t k : order) {
        r0s.push_back(p->leaf_r0[k]);
        ms.push_back(p->leaf_m[k]);
    }
    p->leaf_r0 = r0s;
    p->leaf_m = ms;
}

static void upload_problem_p1(gaca_problem *p);

static void upload_problem(gaca_problem *p) {
    if (p->p1()) {
        upload_problem_p1(p);
        return;
    }
    gaca_context *ctx = p->ctx;
    const int64_t M = p->M;
    // geometry SoA in tree order: 18 arrays of M + 24 arrays (6 points x 4) of M
    const int nsoa = 18 + 24;
    std::vector<double> geo((size_t)nsoa * M);
    double bary[6][3], w6[6];
    triangle6(bary, w6);
    for (int64_t t = 0; t < M; ++t) {
        const int64_t e = p->tree.perm[t];
        const double *v = &p->mesh.vert[9 * e];
        for (int k = 0; k < 9; ++k) geo[(size_t)k * M + t] = v[k];
        for (int k = 0; k < 3; ++k) geo[(size_t)(9 + k) * M + t] = p->mesh.cen[3 * e + k];
        for (int k = 0; k < 3; ++k) geo[(size_t)(12 + k) * M + t] = p->mesh.nrm[3 * e + k];
        geo[(size_t)15 * M + t] = p->mesh.dpl[e];
        geo[(size_t)16 * M + t] = p->mesh.hmax[e];
        geo[(size_t)17 * M + t] = p->mesh.area[e];
        for (int q = 0; q < 6; ++q) {
            for (int k = 0; k < 3; ++k)
                geo[(size_t)(18 + 6 * k + q) * M + t] =
                    bary[q][0] * v[k] + bary[q][1] * v[3 + k] + bary[q][2] * v[6 + k];
            geo[(size_t)(18 + 18 + q) * M + t] = w6[q] * p->mesh.area[e];
        }
    }
    p->d_geo.upload(ctx, geo);
    const double *G = p->d_geo.as<double>();
    GeoDev &g = p->g;
    g.M = M;
    g.T = M;
    const double **fields[18] = {&g.ax, &g.ay, &g.az, &g.bx, &g.by, &g.bz, &g.cx, &g.cy, &g.cz,
                                 &g.xx, &g.xy, &g.xz, &g.nx, &g.ny, &g.nz, &g.d, &g.h, &g.area};
    for (int k = 0; k < 18; ++k) *fields[k] = G + (size_t)k * M;
    g.q6x = G + (size_t)18 * M;
    g.q6y = G + (size_t)24 * M;
    g.q6z = G + (size_t)30 * M;
    g.q6w = G + (size_t)36 * M;
    // FP32 far-rule data for the mixed path: points relative to the centroid, weights
    std::vector<float> geo32((size_t)24 * M);
    for (int64_t t = 0; t < M; ++t)
        for (int q = 0; q < 6; ++q) {
            for (int k = 0; k < 3; ++k)
                geo32[(size_t)(6 * k + q) * M + t] =
                    (float)(geo[(size_t)(18 + 6 * k + q) * M + t] - geo[(size_t)(9 + k) * M + t]);
            geo32[(size_t)(18 + q) * M + t] = (float)geo[(size_t)(36 + q) * M + t];
        }
    p->d_geo32.upload(ctx, geo32);
    const float *G32 = p->d_geo32.as<float>();
    g.q6dx = G32;
    g.q6dy = G32 + (size_t)6 * M;
    g.q6dz = G32 + (size_t)12 * M;
    g.q6wf = G32 + (size_t)18 * M;
    upload_quad(p);
    // permutation
    p->d_perm.upload(ctx, p->tree.perm);
    // near blocks and tier pair lists
    p->nblocks.clear();
    int64_t off = 0;
    std::vector<NearPair> pairs[kNumTiers];
    const bool gal = p->scheme == GACA_GALERKIN_P0;
    for (size_t b = 0; b < p->part.near.size(); ++b) {
        const auto &nb = p->part.near[b];
        NearBlockDev d{(int32_t)nb[0], (int32_t)nb[1], (int32_t)nb[2], (int32_t)nb[3], off};
        p->nblocks.push_back(d);
        off += nb[1] * nb[3] * (int64_t)p->L;
        if (nb[1] > 32767 || nb[3] > 32767)
            throw Error{GACA_ERR_UNSUPPORTED, "near block side above 32767"};
        for (int64_t i = 0; i < nb[1]; ++i)
            for (int64_t j = 0; j < nb[3]; ++j) {
                const int64_t oi = p->tree.perm[nb[0] + i], oj = p->tree.perm[nb[2] + j];
                const int32_t tier =
                    gal ? galerkin_tier(p->mesh, oi, oj) : collocation_tier(p->mesh, oi, oj);
                pairs[tier].push_back(NearPair{(int32_t)b, (int16_t)i, (int16_t)j});
            }
    }
    p->near_elems = off;
    p->d_nblocks.upload(ctx, p->nblocks);
    for (int t = 0; t < kNumTiers; ++t) {
        p->npairs[t] = (int64_t)pairs[t].size();
        p->d_pairs[t].upload(ctx, pairs[t]);
    }
    set_leaves(p);
}

// Geometry of the P1 double layer (layout in GeoDev): triangle arrays in the original
// triangle order, vertex coordinates, patches and vertex ids in the tree order of the
// vertices; one near pair list (the tier is chosen per triangle on the device).
static void upload_problem_p1(gaca_problem *p) {
    gaca_context *ctx = p->ctx;
    const HostMesh &m = p->mesh;
    const int64_t T = m.M, M = p->M;
    double bary[6][3], w6[6];
    triangle6(bary, w6);
    // doubles: 18 triangle arrays + 3 centroids + 18 rule coordinates + 18 weights (per
    // local vertex) of T, then the 3 vertex coordinates of M
    const int ntri_arrays = 18 + 3 + 18 + 18;
    std::vector<double> geo((size_t)ntri_arrays * T + 3 * (size_t)M);
    for (int64_t t = 0; t < T; ++t) {
        const double *v = &m.vert[9 * t];
        for (int k = 0; k < 9; ++k) geo[(size_t)k * T + t] = v[k];
        for (int k = 0; k < 3; ++k) geo[(size_t)(9 + k) * T + t] = m.cen[3 * t + k];
        for (int k = 0; k < 3; ++k) geo[(size_t)(12 + k) * T + t] = m.nrm[3 * t + k];
        geo[(size_t)15 * T + t] = m.dpl[t];
        geo[(size_t)16 * T + t] = m.hmax[t];
        geo[(size_t)17 * T + t] = m.area[t];
        for (int k = 0; k < 3; ++k) geo[(size_t)(18 + k) * T + t] = m.cen[3 * t + k];
        for (int q = 0; q < 6; ++q) {
            for (int k = 0; k < 3; ++k)
                geo[(size_t)(21 + 6 * k + q) * T + t] =
                    bary[q][0] * v[k] + bary[q][1] * v[3 + k] + bary[q][2] * v[6 + k];
            for (int loc = 0; loc < 3; ++loc)
                geo[(size_t)(39 + 6 * loc + q) * T + t] = w6[q] * m.area[t] * bary[q][loc];
        }
    }
    const size_t xo = (size_t)ntri_arrays * T;
    for (int64_t i = 0; i < M; ++i) {
        const int64_t v = p->tree.perm[i];
        for (int k = 0; k < 3; ++k) geo[xo + (size_t)k * M + i] = m.xyz[3 * v + k];
    }
    p->d_geo.upload(ctx, geo);
    const double *G = p->d_geo.as<double>();
    GeoDev &g = p->g;
    g = GeoDev{};
    g.M = M;
    g.T = T;
    const double **fields[18] = {&g.ax, &g.ay, &g.az, &g.bx, &g.by, &g.bz, &g.cx, &g.cy, &g.cz,
                                 &g.tcx, &g.tcy, &g.tcz, &g.nx, &g.ny, &g.nz, &g.d, &g.h, &g.area};
    for (int k = 0; k < 18; ++k) *fields[k] = G + (size_t)k * T;
    g.q6x = G + (size_t)21 * T;
    g.q6y = G + (size_t)27 * T;
    g.q6z = G + (size_t)33 * T;
    g.q6wl = G + (size_t)39 * T;
    g.xx = G + xo;
    g.xy = G + xo + M;
    g.xz = G + xo + 2 * (size_t)M;
    // patches in tree order, triangle vertex ids, vertex id per tree position
    std::vector<std::vector<std::pair<int32_t, int32_t>>> pat(M);
    for (int64_t t = 0; t < T; ++t)
        for (int c = 0; c < 3; ++c) pat[p->inv_perm[m.tri[3 * t + c]]].push_back({(int32_t)t, c});
    p->pptr.assign(M + 1, 0);
    p->ptri.clear();
    p->ploc.clear();
    p->patch_prefix.assign(M + 1, 0.0);
    for (int64_t i = 0; i < M; ++i) {
        std::sort(pat[i].begin(), pat[i].end());
        for (const auto &e : pat[i]) {
            p->ptri.push_back(e.first);
            p->ploc.push_back(e.second);
        }
        if (p->ptri.size() > (size_t)INT32_MAX) throw Error{GACA_ERR_UNSUPPORTED, "P1 patches too large"};
        p->pptr[i + 1] = (int32_t)p->ptri.size();
        p->patch_prefix[i + 1] = p->patch_prefix[i] + (double)pat[i].size();
    }
    const size_t np = p->ptri.size();
    std::vector<int32_t> ints((size_t)(M + 1) + 2 * np + 3 * (size_t)T + (size_t)M);
    size_t o = 0;
    std::copy(p->pptr.begin(), p->pptr.end(), ints.begin());
    o += M + 1;
    std::copy(p->ptri.begin(), p->ptri.end(), ints.begin() + o);
    o += np;
    std::copy(p->ploc.begin(), p->ploc.end(), ints.begin() + o);
    o += np;
    for (int c = 0; c < 3; ++c)
        for (int64_t t = 0; t < T; ++t) ints[o + (size_t)c * T + t] = m.tri[3 * t + c];
    o += 3 * (size_t)T;
    for (int64_t i = 0; i < M; ++i) ints[o + i] = (int32_t)p->tree.perm[i];
    p->d_p1i.upload(ctx, ints);
    const int32_t *I = p->d_p1i.as<int32_t>();
    g.pptr = I;
    g.ptri = I + (M + 1);
    g.ploc = I + (M + 1) + np;
    g.tv0 = I + (M + 1) + 2 * np;
    g.tv1 = g.tv0 + T;
    g.tv2 = g.tv1 + T;
    g.dvid = g.tv2 + T;
    upload_quad(p);
    p->d_perm.upload(ctx, p->tree.perm);
    // near blocks: one pair list; the host counts the quadrature points of every pair with
    // the device's per-triangle rule (algorithmic work of the near field)
    p->nblocks.clear();
    int64_t off = 0;
    std::vector<NearPair> pairs;
    const double nm2 = (double)p->opt.quad_mid * p->opt.quad_mid;
    const double nn2 = (double)p->opt.quad_near * p->opt.quad_near;
    double pts = 0.0;
    for (size_t b = 0; b < p->part.near.size(); ++b) {
        const auto &nb = p->part.near[b];
        NearBlockDev d{(int32_t)nb[0], (int32_t)nb[1], (int32_t)nb[2], (int32_t)nb[3], off};
        p->nblocks.push_back(d);
        off += nb[1] * nb[3] * (int64_t)p->L;
        if (nb[1] > 32767 || nb[3] > 32767)
            throw Error{GACA_ERR_UNSUPPORTED, "near block side above 32767"};
        for (int64_t i = 0; i < nb[1]; ++i) {
            const int64_t vi = p->tree.perm[nb[0] + i];
            const double *x = &m.xyz[3 * vi];
            for (int64_t j = 0; j < nb[3]; ++j) {
                pairs.push_back(NearPair{(int32_t)b, (int16_t)i, (int16_t)j});
                const int64_t tj = nb[2] + j;
                if (p->scheme == GACA_GALERKIN_P1) {
                    // estimate: 36 points per triangle pair of the two patches
                    pts += 36.0 * (p->pptr[nb[0] + i + 1] - p->pptr[nb[0] + i]) * (p->pptr[tj + 1] - p->pptr[tj]);
                    continue;
                }
                for (int32_t e = p->pptr[tj]; e < p->pptr[tj + 1]; ++e) {
                    const int64_t t = p->ptri[e];
                    if (m.tri[3 * t] == vi || m.tri[3 * t + 1] == vi || m.tri[3 * t + 2] == vi) continue;
                    double dv[3];
                    for (int k = 0; k < 3; ++k) dv[k] = x[k] - m.cen[3 * t + k];
                    const double qd = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]) / m.hmax[t];
                    pts += qd >= 4.0 ? 6.0 : (qd >= 2.0 ? nm2 : nn2);
                }
            }
        }
    }
    p->near_elems = off;
    p->p1_near_points = pts;
    p->d_nblocks.upload(ctx, p->nblocks);
    for (int t = 0; t < kNumTiers; ++t) {
        p->npairs[t] = t == 0 ? (int64_t)pairs.size() : 0;
        if (t == 0) p->d_pairs[t].upload(ctx, pairs);
    }
    set_leaves(p);
}

static void upload_freq(gaca_problem *p) {
    std::vector<double> fr(2 * p->L);
    for (int l = 0; l < p->L; ++l) {
        fr[l] = p->s_re[l];
        fr[p->L + l] = p->s_im[l];
    }
    p->d_freq.upload(p->ctx, fr);
    p->f.L = p->L;
    p->f.re = p->d_freq.as<double>();
    p->f.im = p->d_freq.as<double>() + p->L;
    p->f.mirror = p->mirror ? 1 : 0;
    p->f.L_eval = p->mirror ? (p->L + 1) / 2 : p->L;
}

gaca_status gaca_problem_create(gaca_context *ctx, const double *xyz, int64_t nv,
                                const int32_t *tri, int64_t M, const double *s_re,
                                const double *s_im, int32_t L, gaca_scheme scheme,
                                const gaca_options *opt, gaca_problem **out) {
    return guarded([&] {
        REQUIRE(ctx && out, "null context or output");
        REQUIRE(s_re && s_im, "null frequencies");
        REQUIRE(L >= 1 && L <= 1024, "L must be in [1, 1024]");
        REQUIRE(scheme == GACA_COLLOCATION_P0 || scheme == GACA_GALERKIN_P0 ||
                    scheme == GACA_COLLOCATION_P1 || scheme == GACA_GALERKIN_P1, "bad scheme");
        auto p = std::make_unique<gaca_problem>();
        p->attach(ctx);
        if (opt) p->opt = *opt;
        else options_default(&p->opt);
        REQUIRE(p->opt.eta > 0.0, "eta must be > 0");
        REQUIRE(p->opt.eps3d >= 0.0 && p->opt.eps_aca >= 0.0, "tolerances must be >= 0");
        REQUIRE(p->opt.n_duffy >= 1 && p->opt.n_duffy <= 64, "n_duffy out of range");
        REQUIRE(p->opt.n_galerkin >= 1 && p->opt.n_galerkin <= 32, "n_galerkin out of range");
        REQUIRE(p->opt.n_touch >= 1 && p->opt.n_touch <= 32, "n_touch out of range");
        REQUIRE(p->opt.quad_mid >= 1 && p->opt.quad_mid <= 32, "quad_mid out of range");
        REQUIRE(p->opt.quad_near >= 1 && p->opt.quad_near <= 32, "quad_near out of range");
        if (p->opt.autotune_cache) p->autotune_path = p->opt.autotune_cache;
        p->opt.autotune_cache = p->autotune_path.empty() ? nullptr : p->autotune_path.c_str();
        REQUIRE(p->opt.tie >= 0.0 && p->opt.tie < 1.0, "tie out of range");
        ctx->limit = p->opt.max_device_bytes;
        p->scheme = scheme;
        p->mesh.init(xyz, nv, tri, M);
        p->M = M;
        if (scheme == GACA_COLLOCATION_P1 || scheme == GACA_GALERKIN_P1) {
            if (p->opt.precision == GACA_MIXED)
                throw Error{GACA_ERR_UNSUPPORTED, "the P1 operators are built in FP64 only"};
            p1_dofs(p->mesh, p->dofs);
            p->M = nv;
        }
        p->L = L;
        REQUIRE(p->opt.near_aca == 0 || p->opt.near_aca == 1, "near_aca must be 0 or 1");
        if (p->opt.near_aca && L > kNearAcaMaxFreq)
            throw Error{GACA_ERR_UNSUPPORTED, "near_aca supports up to " + std::to_string(kNearAcaMaxFreq) + " frequencies"};
        p->s_re.assign(s_re, s_re + L);
        p->s_im.assign(s_im, s_im + L);
        for (int l = 0; l < L; ++l)
            REQUIRE(std::isfinite(s_re[l]) && std::isfinite(s_im[l]), "non-finite frequency");
        bool mir = true;
        for (int l = 0; l < L; ++l)
            if (!(s_re[L - 1 - l] == s_re[l] && s_im[L - 1 - l] == -s_im[l])) mir = false;
        p->mirror = mir;
        p->tree.build(p->p1() ? p->dofs : p->mesh, p->opt.leaf_size);
        p->part.build(p->tree, p->opt.eta);
        p->inv_perm.assign(p->M, 0);
        for (int64_t t = 0; t < p->M; ++t) p->inv_perm[p->tree.perm[t]] = t;
        GACA_HIP_CHECK(hipSetDevice(ctx->device));
        upload_problem(p.get());
        upload_freq(p.get());
        *out = p.release();
    });
}

gaca_status gaca_problem_destroy(gaca_problem *p) {
    if (!p) return GACA_OK;
    p->destroy_requested = true;
    if (p->nops.load() == 0) delete p;
    return GACA_OK;
}

gaca_status gaca_problem_perm(const gaca_problem *p, int64_t *perm) {
    return guarded([&] {
        REQUIRE(p && perm, "null argument");
        std::copy(p->tree.perm.begin(), p->tree.perm.end(), perm);
    });
}

gaca_status gaca_problem_block_counts(const gaca_problem *p, int64_t *n_far, int64_t *n_near) {
    return guarded([&] {
        REQUIRE(p && n_far && n_near, "null argument");
        *n_far = (int64_t)p->part.far.size();
        *n_near = (int64_t)p->part.near.size();
    });
}

gaca_status gaca_problem_blocks(const gaca_problem *p, int64_t *far4, int64_t *near4) {
    return guarded([&] {
        REQUIRE(p, "null problem");
        if (far4)
            for (size_t b = 0; b < p->part.far.size(); ++b)
                for (int k = 0; k < 4; ++k) far4[4 * b + k] = p->part.far[b][k];
        if (near4)
            for (size_t b = 0; b < p->part.near.size(); ++b)
                for (int k = 0; k < 4; ++k) near4[4 * b + k] = p->part.near[b][k];
    });
}

// ---------------------------------------------------------------------------------------
// far-field build
// Launch class of a far block in the aca phase: faces of kinds 0-2 stay in LDS (R and S,
// up to 128 KB), kind 3 keeps R in HBM.
// Large faces with both sides at most this run as medium faces (see run_far).
constexpr int kMediumSide = 128;

// (The mixed build had FP32 faces of up to 8192 entries in registers too: the faces of 4097
// to 8192 entries run faster on the one-entry-per-thread kernel, as in the FP64 build.)
static int far_kind(int m, int n) {
    const int64_t mn = (int64_t)m * n;
    if (mn <= 1024 && m <= 64 && n <= 64) return 0;
    if (mn <= 2304 && m <= 96 && n <= 96) return 1;
    if (mn <= 4096 && m <= 128 && n <= 128) return 2;
    return 3;
}

// Grow buf to at least need bytes keeping its first `used` bytes (stream-ordered copy).
static void grow_keep(gaca_context *ctx, DevBuf &buf, size_t need, size_t used, hipStream_t st) {
    if (buf.bytes >= need && buf.ptr) return;
    DevBuf nb;
    nb.alloc(ctx, std::max(need, buf.bytes + buf.bytes / 2));
    if (used > 0 && buf.ptr)
        GACA_HIP_CHECK(hipMemcpyAsync(nb.ptr, buf.ptr, std::min(used, buf.bytes),
                                      hipMemcpyDeviceToDevice, st));
    GACA_HIP_CHECK(hipStreamSynchronize(st));
    std::swap(buf.ptr, nb.ptr);
    std::swap(buf.bytes, nb.bytes);
}

// Grow buf to at least need bytes; the contents are not kept.
static void ensure(gaca_context *ctx, DevBuf &buf, size_t need) {
    if (buf.bytes >= need && buf.ptr) return;
    buf.alloc(ctx, std::max(need, buf.bytes + buf.bytes / 2));
}

// Replace buf by a copy holding its first `used` bytes when that frees a useful amount.
static void compact(gaca_context *ctx, DevBuf &buf, size_t used, hipStream_t st);

static void grow_keep(gaca_context *ctx, GrowBuf &buf, size_t need, size_t used, hipStream_t st) {
    buf.grow(ctx, need, used, st);
}

static void compact(gaca_context *ctx, GrowBuf &buf, size_t used, hipStream_t st) {
    if (buf.vmm) {
        buf.shrink(used);
        return;
    }
    compact(ctx, buf.plain, used, st);
    buf.ptr = buf.plain.ptr;
    buf.bytes = buf.plain.bytes;
}

static void compact(gaca_context *ctx, DevBuf &buf, size_t used, hipStream_t st) {
    if (used == 0 || buf.bytes < (64u << 20) || used > buf.bytes / 4 * 3) return;
    DevBuf tight;
    tight.alloc(ctx, used);
    GACA_HIP_CHECK(hipMemcpyAsync(tight.ptr, buf.ptr, used, hipMemcpyDeviceToDevice, st));
    GACA_HIP_CHECK(hipStreamSynchronize(st));
    std::swap(buf.ptr, tight.ptr);
    std::swap(buf.bytes, tight.bytes);
}

// Far field: batches of blocks within the memory budget; in each batch, iterations of the
// four phases over the unfinished blocks until every block has stopped.  The host assigns
// the H / fibre slots of each face and the arena offsets of accepted factors, so storage
// is exact and the layout does not depend on the order in which workgroups run.
static double wall_ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Far field of one operator, or (H of size 2) of the single and double layer operators of
// one collocation problem at once: their blocks are interleaved in one block list, so every
// iteration's launches carry faces of both (each block's kernel in FarBlockDev::kern), and
// the outputs go to each operator's own arenas and tables.
// Mixed-precision scaling geometry of far block b from its cluster boxes: D = x_sigma -
// y_tau (box centres), Dh = fl32(D), d0f = fl32(|D|), kappa = |Dh|^2 - d0f^2 (FP64, then
// FP32) and xs_adj = x_sigma - (D - Dh).
static void set_far_scaling(const gaca_problem *p, int64_t b, FarBlockDev &d) {
    if (p->synthetic || p->part.far_nodes.size() != p->part.far.size()) return;
    const auto &ns = p->tree.nodes[p->part.far_nodes[b][0]];
    const auto &nt = p->tree.nodes[p->part.far_nodes[b][1]];
    double D[3], dd = 0.0;
    for (int k = 0; k < 3; ++k) {
        const double xs = 0.5 * (ns.lo[k] + ns.hi[k]), yt = 0.5 * (nt.lo[k] + nt.hi[k]);
        D[k] = xs - yt;
        dd += D[k] * D[k];
        d.yt[k] = yt;
        d.Dh[k] = (float)D[k];
        d.xs_adj[k] = xs - (D[k] - (double)d.Dh[k]);
    }
    d.d0f = (float)std::sqrt(dd);
    double kap = -(double)d.d0f * (double)d.d0f;
    for (int k = 0; k < 3; ++k) kap += (double)d.Dh[k] * (double)d.Dh[k];
    d.kappa = (float)kap;
}

static void run_far(const std::vector<gaca_hmatrix *> &H, const double2 *dense,
                    const std::function<void()> &main_work) {
    const auto t_entry = std::chrono::steady_clock::now();
    gaca_hmatrix *h = H[0];   // problem, precision and rank cap are common to all of H
    const int nh = (int)H.size();
    gaca_problem *p = h->p;
    gaca_context *ctx = p->ctx;
    const auto &far = p->part.far;
    const int64_t nfar = (int64_t)far.size();
    const int64_t ntot = nh * nfar;   // block gb: operator gb % nh, far block gb / nh
    const int L = p->L;
    const int rcap = h->rcap;
    const bool mixed = h->prec == GACA_MIXED;
    const size_t es = mixed ? sizeof(float2) : sizeof(double2);
    const int PS = far_part_stride(rcap);
    const int fk = nh == 1 ? h->kernel : -1;   // face / tail launch kernel id
    if (nfar == 0) {
        for (gaca_hmatrix *hh : H) {
            hh->nfar = 0;
            hh->meta.clear();
            hh->cmeta.clear();
            hh->cross_off.clear();
            hh->fib_off.clear();
            hh->d_far4.alloc(ctx, 4 * sizeof(int32_t));
        }
        main_work();
        return;
    }
    if (!p->far_streams_ready) {
        {
            std::lock_guard<std::mutex> lk(ctx->stream_mu);
            if (!ctx->stream_pool.empty()) {
                for (int k = 0; k < 4; ++k) p->far_streams[k] = ctx->stream_pool.back()[k];
                ctx->stream_pool.pop_back();
                p->far_streams_ready = true;
            }
        }
        if (!p->far_streams_ready) {
            for (int k = 0; k < 4; ++k)
                GACA_HIP_CHECK(hipStreamCreateWithFlags(&p->far_streams[k], hipStreamNonBlocking));
            p->far_streams_ready = true;
        }
    }
    hipStream_t s0 = p->far_streams[0];
    // the near field first, on the context stream: its kernels run while the host prepares
    // the far field, whose copies and clears go to the far stream (non-blocking, so they do
    // not wait for the near field)
    main_work();
    std::vector<int32_t> far4(4 * nfar);
    for (int64_t b = 0; b < nfar; ++b)
        for (int k = 0; k < 4; ++k) far4[4 * b + k] = (int32_t)far[b][k];
    for (gaca_hmatrix *hh : H) {
        hh->nfar = nfar;
        DevBuf *tabs[5] = {&hh->d_meta, &hh->d_cmeta, &hh->d_cross_off, &hh->d_fib_off, &hh->d_far4};
        const size_t tb[5] = {nfar * sizeof(FarMeta), nfar * rcap * sizeof(CrossMeta),
                              nfar * rcap * sizeof(int64_t), nfar * sizeof(int64_t),
                              far4.size() * sizeof(int32_t)};
        {
            std::lock_guard<std::mutex> lk(p->spare_mu);
            const int k = hh->kernel & 1;
            for (int t = 0; t < 5; ++t)
                if (p->tab_spare[k][t].ptr && p->tab_spare[k][t].bytes == tb[t]) tabs[t]->swap(p->tab_spare[k][t]);
            hh->meta.swap(p->meta_spare[k]);
            hh->cmeta.swap(p->cmeta_spare[k]);
            hh->cross_off.swap(p->coff_spare[k]);
            hh->fib_off.swap(p->foff_spare[k]);
        }
        for (int t = 0; t < 5; ++t)
            if (!tabs[t]->ptr) tabs[t]->alloc(ctx, tb[t]);
        // every entry is overwritten from the device tables when the far field completes
        hh->meta.resize(nfar);
        hh->cmeta.resize(nfar * rcap);
        hh->cross_off.resize(nfar * rcap);
        hh->fib_off.resize(nfar);
        GACA_HIP_CHECK(hipMemcpyAsync(hh->d_far4.ptr, far4.data(), far4.size() * sizeof(int32_t),
                                      hipMemcpyHostToDevice, s0));
    }
    // per-block outputs, indexed by FarBlockDev::out_idx = operator * nfar + far block: the
    // first operator's tables directly, or joint tables split at the end
    DevBuf j_meta, j_cmeta, j_cross_off, j_fib_off;
    if (nh > 1) {
        j_meta.alloc(ctx, ntot * sizeof(FarMeta));
        j_cmeta.alloc(ctx, ntot * rcap * sizeof(CrossMeta));
        j_cross_off.alloc(ctx, ntot * rcap * sizeof(int64_t));
        j_fib_off.alloc(ctx, ntot * sizeof(int64_t));
    }
    DevBuf &o_meta = nh > 1 ? j_meta : h->d_meta, &o_cmeta = nh > 1 ? j_cmeta : h->d_cmeta;
    DevBuf &o_cross_off = nh > 1 ? j_cross_off : h->d_cross_off, &o_fib_off = nh > 1 ? j_fib_off : h->d_fib_off;
    GACA_HIP_CHECK(hipMemsetAsync(o_meta.ptr, 0, ntot * sizeof(FarMeta), s0));
    GACA_HIP_CHECK(hipMemsetAsync(o_cmeta.ptr, 0, ntot * rcap * sizeof(CrossMeta), s0));
    GACA_HIP_CHECK(hipMemsetAsync(o_cross_off.ptr, 0xff, ntot * rcap * sizeof(int64_t), s0));
    GACA_HIP_CHECK(hipMemsetAsync(o_fib_off.ptr, 0xff, ntot * sizeof(int64_t), s0));
    AcaParams P{};
    P.eps = p->opt.eps3d;
    P.eps_aca = p->opt.eps_aca;
    P.tie = p->opt.tie;
    P.delta = p->opt.delta_zero;
    if (mixed) {
        // FP32 faces: the face tolerance, tie window and zero threshold cannot go below
        // what FP32 resolves
        P.eps_aca = std::max(P.eps_aca, 2e-6);
        P.tie = std::max(P.tie, 1e-4);
        P.delta = std::max(P.delta, 1e-6);
    }
    for (gaca_hmatrix *hh : H) hh->eps_aca_used = P.eps_aca;
    P.rcap = rcap;
    P.kernel = fk;
    P.zero_batch = p->opt.zero_rows_batch != 0;
    P.recompress = p->opt.recompress != 0;
    P.pivot_index = p->opt.pivot_estimate != 0;
    const bool recomp = P.recompress != 0;

    // block descriptors, launch classes and memory estimates
    std::vector<FarBlockDev> desc(ntot);
    std::vector<int> kind(ntot);
    // memory estimate of a block in a batch with rg faces per block (pool slots, fibres and
    // Gram rows, current factors, expand partials, state)
    auto est_of = [&](int64_t gb, double rg) {
        const double m = (double)desc[gb].m, n = (double)desc[gb].n, mn = m * n;
        const double rho_max = std::min(m, n);
        const double tiles = far_kind((int)m, (int)n) == 3 ? std::ceil(m / 32.0) * std::ceil(n / 32.0) : 1.0;
        return 2.0 * rho_max * (m + n) * es + (rg + 1) * mn * es + rg * (double)(L + rcap) * 16 +
               tiles * PS * 8 + sizeof(FarStateDev) + sizeof(FarBlockDev) + rcap * 32.0 + L + 64;
    };
    // faces per block of the memory estimate: what the last build of this operator kind
    // stored (with a quarter added), else a generous first guess
    const int fpb_slot = nh > 1 ? 6 : std::min(std::max(h->kernel, 0), 5);   // kernel id 0-5
    double rguess = p->faces_per_block[fpb_slot] > 0 ? std::min((double)rcap, p->faces_per_block[fpb_slot])
                                                     : std::min(rcap, 24);
    double factor_guess = 0.0;
    for (int64_t b = 0; b < nfar; ++b) {
        const int m = (int)far[b][1], n = (int)far[b][3];
        if (m > kFarMaxRows || n > kFarMaxRows)
            throw Error{GACA_ERR_UNSUPPORTED, "far block with more than 8192 rows or columns"};
        int rho_max = std::min(m, n);
        if (p->opt.max_face_rank > 0) rho_max = std::min(rho_max, p->opt.max_face_rank);
        FarBlockDev d{};
        d.r0 = (int32_t)far[b][0];
        d.m = m;
        d.c0 = (int32_t)far[b][2];
        d.n = n;
        d.rho_max = rho_max;
        d.out_idx = (int32_t)b;   // operator 0; copies below for the others
        set_far_scaling(p, b, d);
        for (int w = 0; w < nh; ++w) {
            FarBlockDev dw = d;
            dw.out_idx = (int32_t)(w * nfar + b);
            dw.kern = H[w]->kernel;
            dw.which = w;
            desc[nh * b + w] = dw;
            kind[nh * b + w] = far_kind(m, n);
        }
        const double mn = (double)m * n;
        // first guess of the factor storage (the arena grows by half when it runs short)
        factor_guess += std::min(mn * L, (double)std::min(rcap, 8) * std::min(rho_max, 16) * (m + n));
    }
    // blocks enter the batches by size, the largest first (ties in partition order): a batch
    // iterates until its block with the most crosses is done, and the large blocks, which
    // take the most crosses and the longest face ACAs, then share a few batches instead of
    // drawing out every batch.  The result tables are indexed by out_idx, so the order
    // changes no result.
    {
        std::vector<int64_t> ord(nfar);
        std::iota(ord.begin(), ord.end(), (int64_t)0);
        std::stable_sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) {
            return (int64_t)far[x][1] * far[x][3] > (int64_t)far[y][1] * far[y][3];
        });
        std::vector<FarBlockDev> dsort(ntot);
        std::vector<int> ksort(ntot);
        for (int64_t i = 0; i < nfar; ++i)
            for (int w = 0; w < nh; ++w) {
                dsort[nh * i + w] = desc[nh * ord[i] + w];
                ksort[nh * i + w] = kind[nh * ord[i] + w];
            }
        desc.swap(dsort);
        kind.swap(ksort);
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        free_b = (size_t)p->opt.batch_bytes;
    }

    // the aca phase of kind k runs on ks[k] (kind 3, the large faces, on the main far stream)
    const hipStream_t ks[4] = {p->far_streams[3], p->far_streams[2], p->far_streams[1], s0};
    enum { EV_BEGIN, EV_END, EV_F0, EV_F1, EV_K0, EV_K1, EV_K2, EV_K3, EV_S0, EV_S1, EV_S2, EV_S3, EV_J, EV_X,
           EV_T, EV_C, EV_P0, EV_P2, EV_N };
    hipEvent_t ev[EV_N];
    for (auto &e : ev) GACA_HIP_CHECK(hipEventCreate(&e));
    struct EvGuard {
        hipEvent_t *e;
        ~EvGuard() {
            for (int i = 0; i < EV_N; ++i) (void)hipEventDestroy(e[i]);
        }
    } ev_guard{ev};
    GACA_HIP_CHECK(hipEventRecord(ev[EV_BEGIN], s0));
    const double ms_setup = wall_ms_since(t_entry);
    double ms_wait = 0.0;   // host time blocked on the per-iteration status read-back
    double ms_prep = 0.0, ms_launch = 0.0;   // host time preparing / enqueuing iterations
    g_mem_verbose = p->opt.verbose;
    const int64_t mem_ns0 = g_mem_ns.load(), mem_calls0 = g_mem_calls.load();

    FarScratch &W = p->fsc;
    size_t arena_used[2] = {0, 0}, fib_used[2] = {0, 0};
    // a spare arena (the same problem's last build needed about its size) is taken as it is
    // and grows only when this build outgrows it; otherwise a new one starts at `need`.  The
    // spare of the same operator (slot kernel & 1) is tried first, so that the single and
    // double layer do not trade arenas of slightly different sizes from build to build (each
    // trade maps and unmaps chunks)
    auto start_arena = [&](GrowBuf &dst, GrowBuf *spare, int pref, size_t need) {
        {
            std::lock_guard<std::mutex> lk(p->spare_mu);
            for (int t = 0; t < 2 && !dst.ptr; ++t) {
                const int k = t == 0 ? pref : 1 - pref;
                if (spare[k].ptr) dst.swap(spare[k]);
            }
        }
        if (!dst.ptr) dst.start(ctx, need);
    };
    for (gaca_hmatrix *hh : H) {
        start_arena(hh->d_arena, p->spare_arena, hh->kernel & 1, (size_t)std::max(1.0e5, factor_guess) * es);
        start_arena(hh->d_fib, p->spare_fib, hh->kernel & 1,
                    (size_t)std::max<int64_t>(1024, nfar * (int64_t)std::min(rcap, 16) * L) * sizeof(double2));
    }
    // algorithmic work model (flops; a complex multiply-add is 8): per quadrature point x
    // frequency the single layer costs 105 (distance 8, sqrt 13, exp 31, sincos 36,
    // 1/(4 pi r) 8, weight and accumulation 9), the double layer 113
    auto f_eval_of = [&](int kern) {
        return dense ? 0.0 : (kern == 1 || kern == 3 || kern == 5 ? 113.0 : 105.0);
    };
    // quadrature points per entry: 6 (collocation), 36 (Galerkin), 6 per triangle of the
    // column vertex's patch (P1; the block's mean over its columns)
    auto qpe_of = [&](const FarBlockDev &d) {
        if (h->kernel == 3)
            return 6.0 * (p->patch_prefix[d.c0 + d.n] - p->patch_prefix[d.c0]) / std::max(1, d.n);
        if (h->kernel >= 4)   // 6 x 6 points per pair of triangles of the two patches
            return 36.0 * (p->patch_prefix[d.r0 + d.m] - p->patch_prefix[d.r0]) / std::max(1, d.m) *
                   (p->patch_prefix[d.c0 + d.n] - p->patch_prefix[d.c0]) / std::max(1, d.n);
        return h->kernel == 2 ? 36.0 : 6.0;
    };
    double ms_phase[4] = {0, 0, 0, 0}, ms_kind[4] = {0, 0, 0, 0}, fl_phase[4] = {0, 0, 0, 0};
    double by_phase[4] = {0, 0, 0, 0};   // algorithmic HBM bytes of the face and expand phases
    const double fe_bytes = mixed ? 8.0 : 16.0;   // one face element
    double fl_kind[4] = {0, 0, 0, 0};
    int launches_kind[4] = {0, 0, 0, 0};
    // faces with a side above kMediumSide by kernel path (0 general, 1 one entry per thread,
    // 2 several entries per thread): device time, launches, algorithmic flops
    double ms_path[3] = {0, 0, 0}, fl_path[3] = {0, 0, 0};
    int launches_path[3] = {0, 0, 0};
    int launches_phase[4] = {0, 0, 0, 0};
    int iters_max = 0, n_launch = 0;
    double evals = 0.0;

    if (recomp) ensure(ctx, W.rec_ws, (size_t)kRecSlots * kRecSlot * sizeof(double2));
    // batches of consecutive blocks (in the size order above) whose estimate fits the memory
    // free at their start; the faces-per-block guess of the estimate follows what the
    // previous batches used
    for (int64_t bnext = 0; bnext < ntot;) {
        double budget = 0.0, rest = 0.0, fb_all = 0.0;
        {
            size_t fb = 0, tb = 0;
            if (hipMemGetInfo(&fb, &tb) != hipSuccess) {
                (void)hipGetLastError();
                fb = (size_t)p->opt.batch_bytes;
            }
            // the pools held from the previous batch are reused
            fb += W.hpool.bytes + W.fgpool.bytes + W.uw.bytes + W.part.bytes;
            budget = std::max(64.0 * (1 << 20), std::min((double)p->opt.batch_bytes, 0.5 * (double)fb));
            // the remaining blocks go as one batch when they fit in 60 % of the free memory:
            // one batch saves the second batch's iterations, while several larger batches
            // would leave too little memory between them to keep the pools mapped
            for (int64_t gb = bnext; gb < ntot; ++gb) rest += est_of(gb, rguess);
            fb_all = (double)fb;
            if (rest <= std::min((double)p->opt.batch_bytes, 0.6 * (double)fb)) budget = std::max(budget, rest);
        }
        int64_t blast = bnext;
        double acc = 0.0;
        while (blast < ntot) {
            const double e = est_of(blast, rguess);
            if (blast > bnext && acc + e > budget) break;
            acc += e;
            ++blast;
        }
        if (p->opt.verbose) {
            std::fprintf(stderr, "gaca far field: batch of blocks %lld..%lld of %lld: estimate %.2f GB (all "
                         "remaining blocks %.2f GB) at %.1f faces per block, budget %.2f GB of %.2f GB free\n",
                         (long long)bnext, (long long)blast, (long long)ntot, acc / 1e9, rest / 1e9, rguess,
                         budget / 1e9, fb_all / 1e9);
            std::fflush(stderr);
        }
        const std::pair<int64_t, int64_t> bt{bnext, blast};
        bnext = blast;
        const int64_t base = bt.first;
        const int nb = (int)(bt.second - bt.first);
        std::vector<FarBlockDev> bdesc(desc.begin() + bt.first, desc.begin() + bt.second);
        int64_t uw_total = 0;
        for (auto &d : bdesc) {
            d.uw_off = uw_total;
            uw_total += (int64_t)d.rho_max * (d.m + d.n);
        }
        // upload without reallocating: a free would wait for the near field running beside
        ensure(ctx, W.blk, bdesc.size() * sizeof(FarBlockDev));
        W.h_blk.ensure(bdesc.size() * sizeof(FarBlockDev));
        std::memcpy(W.h_blk.ptr, bdesc.data(), bdesc.size() * sizeof(FarBlockDev));
        GACA_HIP_CHECK(hipMemcpyAsync(W.blk.ptr, W.h_blk.ptr, bdesc.size() * sizeof(FarBlockDev),
                                      hipMemcpyHostToDevice, s0));
        ensure(ctx, W.state, nb * sizeof(FarStateDev));
        ensure(ctx, W.coef, (size_t)nb * rcap * sizeof(double2));
        ensure(ctx, W.hs, (size_t)nb * rcap * sizeof(int64_t));
        ensure(ctx, W.fs, (size_t)nb * rcap * sizeof(int64_t));
        ensure(ctx, W.usedk, (size_t)nb * L);
        // two slots of U, W scratch, alternating by iteration: the copy of the factors
        // accepted in one iteration reads its slot while the next iteration's face ACAs
        // write the other
        ensure(ctx, W.uw, 2 * (size_t)std::max<int64_t>(uw_total, 1) * es);
        ensure(ctx, W.act, nb * sizeof(FarActive));
        ensure(ctx, W.status, nb * 2 * sizeof(int32_t));
        ensure(ctx, W.copies, nb * sizeof(FarCopy));
        ensure(ctx, W.gathers, nb * sizeof(FarGather));
        W.h_act.ensure(nb * sizeof(FarActive));
        W.h_status.ensure(nb * 2 * sizeof(int32_t));
        W.h_copies.ensure(nb * sizeof(FarCopy));
        W.h_gathers.ensure(nb * sizeof(FarGather));
        GACA_HIP_CHECK(hipMemsetAsync(W.state.ptr, 0, nb * sizeof(FarStateDev), s0));
        GACA_HIP_CHECK(hipMemsetAsync(W.usedk.ptr, 0, (size_t)nb * L, s0));
        std::vector<int32_t> ell_h(nb, 0);
        std::vector<int64_t> hcur(nb, -1), fcur(nb, -1);
        std::vector<int> active(nb);
        std::iota(active.begin(), active.end(), 0);
        std::vector<FarCopy> pending;
        int64_t hused = 0, fused = 0;
        int iter = 0;
        bool copy_ev = false;   // ev[EV_C] marks the end of the last copy launched on ks[0]

        auto batch_dev = [&](int slot) {
            FarBatchDev bd{};
            bd.blk = W.blk.as<FarBlockDev>();
            bd.st = W.state.as<FarStateDev>();
            bd.coef = W.coef.as<double2>();
            bd.hs = W.hs.as<int64_t>();
            bd.fs = W.fs.as<int64_t>();
            bd.usedk = W.usedk.as<unsigned char>();
            bd.hpool = W.hpool.ptr;
            bd.fgpool = W.fgpool.as<double2>();
            bd.uw = static_cast<unsigned char *>(W.uw.ptr) + (size_t)slot * std::max<int64_t>(uw_total, 1) * es;
            bd.part = W.part.as<double>();
            bd.map_chunk = W.map_chunk.as<int32_t>();
            bd.map_tile = W.map_tile.as<int32_t>();
            bd.status = W.status.as<int32_t>();
            bd.meta = o_meta.as<FarMeta>();
            bd.cmeta = o_cmeta.as<CrossMeta>();
            bd.dense = dense;
            bd.mixed = mixed ? 1 : 0;
            bd.rcap = rcap;
            bd.L = L;
            return bd;
        };
        // factors of the crosses accepted in the last iteration -> arena, one workgroup per
        // kFarCopyChunk elements; returns whether a copy was launched on stream cs
        std::vector<FarCopy> chunks;
        auto flush_copies = [&](hipStream_t cs) {
            if (pending.empty()) return false;
            // the copy list buffers are reused: the last copy (one iteration ago) has read them
            if (copy_ev) GACA_HIP_CHECK(hipEventSynchronize(ev[EV_C]));
            chunks.clear();
            for (const FarCopy &c : pending) {
                const int64_t tot = (int64_t)c.rho * (bdesc[c.b].m + bdesc[c.b].n);
                const int64_t nch = std::max<int64_t>(1, (tot + kFarCopyChunk - 1) / kFarCopyChunk);
                for (int64_t k = 0; k < nch; ++k) {
                    FarCopy x = c;
                    x.chunk = (int32_t)k;
                    chunks.push_back(x);
                }
            }
            ensure(ctx, W.copies, chunks.size() * sizeof(FarCopy));
            W.h_copies.ensure(chunks.size() * sizeof(FarCopy));
            std::memcpy(W.h_copies.ptr, chunks.data(), chunks.size() * sizeof(FarCopy));
            GACA_HIP_CHECK(hipMemcpyAsync(W.copies.ptr, W.h_copies.ptr, chunks.size() * sizeof(FarCopy),
                                          hipMemcpyHostToDevice, cs));
            void *const arenas[2] = {h->d_arena.ptr, H[nh - 1]->d_arena.ptr};
            // the pending crosses were accepted in the previous iteration: its U, W slot
            launch_far_copy(batch_dev((iter - 1) & 1), W.copies.as<FarCopy>(), (int)chunks.size(), arenas,
                            o_cross_off.as<int64_t>(), cs);
            GACA_HIP_CHECK(hipGetLastError());
            ++n_launch;
            pending.clear();
            return true;
        };

        // kind 3 first (large faces with a side above kMediumSide before the medium ones),
        // then 2, 1, 0; larger faces first within a class
        auto big = [&](int x) { return std::max(bdesc[x].m, bdesc[x].n) > kMediumSide; };
        // large-face kernel path of a big face: 0 general (several entries per thread
        // beyond the register paths), 2 several entries per thread, 1 one entry per thread
        const int tlx = p->opt.threads_large > 0 ? p->opt.threads_large : 512;
        auto path = [&](int x) {
            const int side = std::max(bdesc[x].m, bdesc[x].n);
            if (side <= tlx) return 1;
            return (tlx == 512 && side <= kFarMultiE * 512) ? 2 : 0;
        };
        // one-entry faces with sides <= 256 under a larger workgroup size run with 256
        // threads (two faces per CU) on the class-1 stream, beside the larger faces
        auto small_big = [&](int x) {
            return tlx > 256 && path(x) == 1 && std::max(bdesc[x].m, bdesc[x].n) <= 256;
        };
        auto prank = [&](int x) {
            const int pth = path(x);
            return pth == 0 ? 0 : pth == 2 ? 1 : small_big(x) ? 3 : 2;
        };
        // launch class of a block's face ACA (the stream it runs on)
        auto aca_class = [&](int x) {
            const int kd = kind[base + x];
            if (kd != 3) return kd;
            return !big(x) ? 2 : small_big(x) ? 1 : 3;
        };
        {
            // launch order as one key per block: class (3 first), then for kind 3 the big
            // faces first and among them the path rank, then m n descending; a stable sort
            // keeps the block order among equal keys
            std::vector<int64_t> okey(nb);
            for (int x = 0; x < nb; ++x) {
                const int kd = kind[base + x];
                const bool bg = kd == 3 && big(x);
                const int64_t mn = (int64_t)bdesc[x].m * bdesc[x].n;
                okey[x] = ((int64_t)(3 - kd) << 40) | ((int64_t)(kd == 3 && !bg) << 36) |
                          ((int64_t)(bg ? prank(x) : 0) << 32) | ((int64_t)0xFFFFFFFF - mn);
            }
            std::stable_sort(active.begin(), active.end(), [&](int x, int y) { return okey[x] < okey[y]; });
        }
        while (!active.empty()) {
            const auto t_it = std::chrono::steady_clock::now();
            // slots of this iteration's faces (a zero face keeps its slots for the next one)
            const int64_t hprev = hused, fprev = fused;
            for (int lb : active) {
                const FarBlockDev &d = bdesc[lb];
                if (hcur[lb] < 0) {
                    hcur[lb] = hused;
                    hused += (int64_t)d.m * d.n;
                }
                if (fcur[lb] < 0) {
                    fcur[lb] = fused;
                    fused += L + rcap;
                }
            }
            if (iter == 0) {
                // first guess of the pool sizes (rguess faces per block), kept by the problem
                // across builds; both grow in place when they run short
                double hg = 0.0;
                for (int lb = 0; lb < nb; ++lb) hg += (double)bdesc[lb].m * bdesc[lb].n;
                const double hcap = std::min((rguess + 1) * hg, std::max((double)hused, 0.3 * free_b / es));
                grow_keep(ctx, W.hpool, (size_t)std::max((double)hused, hcap) * es, 0, s0);
                grow_keep(ctx, W.fgpool, (size_t)(nb * (rguess + 1)) * (L + rcap) * sizeof(double2), 0, s0);
            }
            grow_keep(ctx, W.hpool, (size_t)hused * es, (size_t)hprev * es, s0);
            grow_keep(ctx, W.fgpool, (size_t)fused * sizeof(double2), (size_t)fprev * sizeof(double2), s0);
            // the list is in launch order (sorted once before the first iteration; finished
            // blocks leave in order)
            int nbig = 0, nsb = 0, npath[3] = {0, 0, 0};
            while (nbig < (int)active.size() && kind[base + active[nbig]] == 3 && big(active[nbig])) {
                const int x = active[nbig++];
                if (small_big(x)) ++nsb;
                else ++npath[path(x)];
            }
            const int nact = (int)active.size();
            ms_prep += wall_ms_since(t_it);
            const auto t_launch = std::chrono::steady_clock::now();
            FarActive *ha = W.h_act.as<FarActive>();
            int64_t nchunk = 0, ntile = 0;
            int cnt[4] = {0, 0, 0, 0};
            double fl_face = 0.0, by_face = 0.0;
            for (int a = 0; a < nact; ++a) {
                const int lb = active[a];
                const FarBlockDev &d = bdesc[lb];
                const int kd = kind[base + lb];
                const int64_t mn = (int64_t)d.m * d.n;
                FarActive A{};
                A.b = lb;
                A.hslot = hcur[lb];
                A.fgslot = fcur[lb];
                A.chunk0 = nchunk;
                nchunk += (mn + kFarChunk - 1) / kFarChunk;
                A.tile0 = ntile;
                // with recompression every face is expanded again from its new factors
                A.ntile = (kd == 3 || recomp) ? ((d.m + kFarTile - 1) / kFarTile) * ((d.n + kFarTile - 1) / kFarTile) : 0;
                ntile += A.ntile;
                cnt[kd]++;
                ha[a] = A;
            }
            // small faces: one partial row each (their Gram row), after the expand tiles
            if (!recomp)
                for (int a = cnt[3]; a < nact; ++a) ha[a].tile0 = ntile + (a - cnt[3]);
            const int64_t nparts = recomp ? ntile : ntile + (nact - cnt[3]);
            ensure(ctx, W.map_chunk, (size_t)std::max<int64_t>(nchunk, 1) * sizeof(int32_t));
            ensure(ctx, W.map_tile, (size_t)std::max<int64_t>(ntile, 1) * sizeof(int32_t));
            ensure(ctx, W.part, (size_t)std::max<int64_t>(nparts, 1) * PS * sizeof(double));
            GACA_HIP_CHECK(hipMemcpyAsync(W.act.ptr, W.h_act.ptr, nact * sizeof(FarActive),
                                          hipMemcpyHostToDevice, s0));
            const FarBatchDev bd = batch_dev(iter & 1);
            const FarActive *dact = W.act.as<FarActive>();
            const int nlarge = recomp ? nact : cnt[3];
            // act is ordered kind 3, 2, 1, 0
            const int first[4] = {cnt[3] + cnt[2] + cnt[1], cnt[3] + cnt[2], cnt[3], 0};
            launch_far_map(bd, dact, nact, nlarge, s0);
            GACA_HIP_CHECK(hipEventRecord(ev[EV_F0], s0));
            launch_far_face(fk, p->g, p->f, bd, dact, nchunk, s0);
            GACA_HIP_CHECK(hipEventRecord(ev[EV_F1], s0));
            // work model of the face phase, while the face kernel runs
            for (int a = 0; a < nact; ++a) {
                const int lb = active[a];
                const FarBlockDev &d = bdesc[lb];
                const double mn = (double)d.m * d.n, qpe = qpe_of(d);
                evals += mn * qpe;
                fl_face += mn * (qpe * f_eval_of(d.kern) + 8.0 * ell_h[lb]);
                // the previous faces read once, the new face written once
                by_face += mn * (ell_h[lb] + 1.0) * fe_bytes;
            }
            for (int k = 0; k < 3; ++k) GACA_HIP_CHECK(hipStreamWaitEvent(ks[k], ev[EV_F1], 0));
            // this iteration's ACAs write the U, W slot that the previous iteration's copy
            // reads (on ks[0], in order before the class-0 launches)
            if (copy_ev)
                for (int k = 1; k < 4; ++k) GACA_HIP_CHECK(hipStreamWaitEvent(ks[k], ev[EV_C], 0));
            // large faces: 512 threads and ~104 KB of LDS history, one face per CU (the
            // longest face bounds the phase); medium faces (sides <= kMediumSide) 256 threads
            // and 32 KB, several per CU, on the kind-2 stream, so that they do not hold whole
            // CUs against the small-face kinds
            int tl = p->opt.threads_large;
            if (tl <= 0) tl = 512;
            const int ts = p->opt.threads_small;
            // class k's launches run between EV_S0 + k and EV_K0 + k on ks[k] (after its waits)
            for (int k = 0; k < 4; ++k) GACA_HIP_CHECK(hipEventRecord(ev[EV_S0 + k], ks[k]));
            int nl = 0;
            for (int k = 3; k >= 0; --k) {
                if (cnt[k] == 0) continue;
                if (k == 3) {
                    // big faces by path (general, several entries, one entry per thread),
                    // one after the other on the kind-3 stream
                    launch_far_aca(0, tl, P, bd, dact, npath[0], ks[3]);
                    GACA_HIP_CHECK(hipEventRecord(ev[EV_P0], ks[3]));
                    launch_far_aca(2, tl, P, bd, dact + npath[0], npath[2], ks[3]);
                    GACA_HIP_CHECK(hipEventRecord(ev[EV_P2], ks[3]));
                    launch_far_aca(1, tl, P, bd, dact + npath[0] + npath[2], npath[1], ks[3]);
                    launch_far_aca(1, 256, P, bd, dact + npath[0] + npath[2] + npath[1], nsb, ks[1]);
                    launch_far_aca(1, 256, P, bd, dact + nbig, cnt[3] - nbig, ks[2]);
                    nl += (npath[0] > 0) + (npath[2] > 0) + (npath[1] > 0) + (nsb > 0) + (cnt[3] > nbig);
                    continue;
                }
                if (k == 0 && ts <= 64) {
                    // one wave per face: faces with m n <= 576 (after the larger ones) hold
                    // nine register entries per lane instead of sixteen
                    int a = first[0];
                    while (a < first[0] + cnt[0] && (int64_t)bdesc[ha[a].b].m * bdesc[ha[a].b].n > 576) ++a;
                    launch_far_aca_small(1024, 64, P, bd, dact + first[0], a - first[0], ks[0]);
                    launch_far_aca_small(576, 64, P, bd, dact + a, first[0] + cnt[0] - a, ks[0]);
                    nl += (a > first[0]) + (a < first[0] + cnt[0]);
                } else {
                    const int mnmax = k == 0 ? 1024 : k == 1 ? 2304 : 4096;
                    launch_far_aca_small(mnmax, k == 0 ? ts : k == 1 ? 256 : 512, P, bd, dact + first[k],
                                         cnt[k], ks[k]);
                    ++nl;
                }
                if (!recomp) {
                    launch_far_gram_small(bd, dact + first[k], cnt[k], ks[k]);
                    ++nl;
                }
            }
            GACA_HIP_CHECK(hipGetLastError());
            for (int k = 0; k < 4; ++k) GACA_HIP_CHECK(hipEventRecord(ev[EV_K0 + k], ks[k]));
            for (int k = 0; k < 3; ++k) GACA_HIP_CHECK(hipStreamWaitEvent(s0, ev[EV_K0 + k], 0));
            GACA_HIP_CHECK(hipEventRecord(ev[EV_J], s0));
            // the factors accepted in the previous iteration (its U, W slot) -> arena, on ks[0]
            // after the class-0 ACAs: the copy runs beside the large-face ACAs (latency bound)
            // instead of the face kernel, and nothing on s0 waits for it
            if (flush_copies(ks[0])) {
                GACA_HIP_CHECK(hipEventRecord(ev[EV_C], ks[0]));
                copy_ev = true;
            }
            if (recomp) {
                launch_far_recompress(P, bd, dact, nact, W.rec_ws.as<double2>(), kRecSlots, s0);
                ++n_launch;
            }
            launch_far_expand(bd, dact, ntile, s0);
            GACA_HIP_CHECK(hipEventRecord(ev[EV_X], s0));
            launch_far_tail(fk, p->g, p->f, P, bd, dact, nact, nlarge, s0);
            GACA_HIP_CHECK(hipGetLastError());
            GACA_HIP_CHECK(hipEventRecord(ev[EV_T], s0));
            ms_launch += wall_ms_since(t_launch);
            GACA_HIP_CHECK(hipMemcpyAsync(W.h_status.ptr, W.status.ptr, nact * 2 * sizeof(int32_t),
                                          hipMemcpyDeviceToHost, s0));
            {
                const auto tw = std::chrono::steady_clock::now();
                GACA_HIP_CHECK(hipStreamSynchronize(s0));
                ms_wait += wall_ms_since(tw);
            }
            n_launch += 3 + nl + (ntile > 0);
            auto elapsed = [&](int x, int y) {
                float ms = 0.0f;
                GACA_HIP_CHECK(hipEventElapsedTime(&ms, ev[x], ev[y]));
                return (double)ms;
            };
            ms_phase[0] += elapsed(EV_F0, EV_F1);
            ms_phase[1] += elapsed(EV_F1, EV_J);
            ms_phase[2] += elapsed(EV_J, EV_X);
            ms_phase[3] += elapsed(EV_X, EV_T);
            // launch classes by stream: 0, 1 (with the large faces of sides <= 256 when the
            // large workgroup size is above 256), 2 (kind 2 and the medium large faces), 3 (the
            // other large faces, sides above kMediumSide)
            const int ccls[4] = {cnt[0], cnt[1] + nsb, cnt[2] + cnt[3] - nbig, nbig - nsb};
            for (int k = 0; k < 4; ++k)
                if (ccls[k]) {
                    ms_kind[k] += elapsed(EV_S0 + k, EV_K0 + k);
                    launches_kind[k] += 1;
                }
            if (nbig > nsb) {
                // the path launches follow each other on ks[3]: path 0, path 2, path 1
                if (npath[0]) { ms_path[0] += elapsed(EV_S0 + 3, EV_P0); launches_path[0] += 1; }
                if (npath[2]) { ms_path[2] += elapsed(EV_P0, EV_P2); launches_path[2] += 1; }
                if (npath[1]) { ms_path[1] += elapsed(EV_P2, EV_K0 + 3); launches_path[1] += 1; }
            }
            launches_phase[0] += 1;
            launches_phase[1] += nl;
            launches_phase[2] += ntile > 0;
            launches_phase[3] += 1;
            fl_phase[0] += fl_face;
            by_phase[0] += by_face;
            // status: accepted crosses get arena space, finished blocks leave
            const int32_t *hs_ = W.h_status.as<int32_t>();
            std::vector<int> next;
            next.reserve(nact);
            const size_t arena_before[2] = {arena_used[0], arena_used[1]};
            for (int a = 0; a < nact; ++a) {
                const int lb = ha[a].b;
                const FarBlockDev &d = bdesc[lb];
                const int code = hs_[2 * a], rho = hs_[2 * a + 1];
                const double mn = (double)d.m * d.n;
                const int ell = ell_h[lb];
                const int kd = kind[base + lb];
                if (code & 1) {
                    FarCopy c{};
                    c.b = lb;
                    c.p = ell;
                    c.rho = rho;
                    c.which = d.which;
                    c.off = (int64_t)arena_used[d.which];
                    arena_used[d.which] += (size_t)rho * (d.m + d.n);
                    pending.push_back(c);
                    ell_h[lb] = ell + 1;
                    hcur[lb] = -1;
                    fcur[lb] = -1;
                    // face ACA: kind 3 corrects rows / columns from the factor history and
                    // forms the cross terms of |S|^2, 2 (m + n) q complex MACs at step q; the
                    // LDS kinds update R and S in place (2 m n per step) and form the Gram row
                    if (kd == 3) {
                        const double f = 8.0 * (d.m + d.n) * (double)rho * (rho - 1.0);
                        fl_phase[1] += f;
                        const int ac = aca_class(lb);
                        fl_kind[ac] += f;
                        if (ac == 3) fl_path[path(lb)] += f;
                        fl_phase[2] += 8.0 * mn * (rho + ell);
                        // U, W read, H_l written, the previous faces read once (Gram row)
                        by_phase[2] += ((double)rho * (d.m + d.n) + mn * (ell + 1.0)) * fe_bytes;
                    } else {
                        const double f = 8.0 * mn * (2.0 * rho + ell);
                        fl_phase[1] += f;
                        fl_kind[kd] += f;
                    }
                    const double qpe = qpe_of(d);
                    fl_phase[3] += (double)L * qpe * f_eval_of(d.kern) + 16.0 * L * ell + 8.0 * (ell + 1.0) * (ell + 1.0);
                    evals += (double)L * qpe;
                } else {
                    fl_phase[3] += 8.0 * (double)ell * ell;
                }
                if (!(code & 2)) next.push_back(lb);
            }
            for (int w = 0; w < nh; ++w)
                if (arena_used[w] > H[w]->d_arena.bytes / es) {
                    // the copy on ks[0] may still write the arena
                    if (copy_ev) GACA_HIP_CHECK(hipEventSynchronize(ev[EV_C]));
                    grow_keep(ctx, H[w]->d_arena, arena_used[w] * es, arena_before[w] * es, s0);
                }
            active.swap(next);
            ++iter;
        }
        if (copy_ev) GACA_HIP_CHECK(hipStreamWaitEvent(s0, ev[EV_C], 0));
        flush_copies(s0);
        // fibres of the batch -> fibre arena, contiguous per block
        std::vector<FarGather> gth;
        const size_t fib_before[2] = {fib_used[0], fib_used[1]};
        for (int lb = 0; lb < nb; ++lb) {
            FarGather g{};
            g.b = lb;
            g.rank = ell_h[lb];
            g.which = bdesc[lb].which;
            g.off = (int64_t)fib_used[g.which];
            fib_used[g.which] += (size_t)ell_h[lb] * L;
            gth.push_back(g);
        }
        for (int w = 0; w < nh; ++w)
            grow_keep(ctx, H[w]->d_fib, std::max<size_t>(fib_used[w], 1) * sizeof(double2),
                      fib_before[w] * sizeof(double2), s0);
        std::memcpy(W.h_gathers.ptr, gth.data(), gth.size() * sizeof(FarGather));
        GACA_HIP_CHECK(hipMemcpyAsync(W.gathers.ptr, W.h_gathers.ptr, gth.size() * sizeof(FarGather),
                                      hipMemcpyHostToDevice, s0));
        double2 *const fibs[2] = {h->d_fib.as<double2>(), H[nh - 1]->d_fib.as<double2>()};
        launch_far_gather(batch_dev(0), W.gathers.as<FarGather>(), nb, fibs, o_fib_off.as<int64_t>(), s0);
        GACA_HIP_CHECK(hipGetLastError());
        ++n_launch;
        GACA_HIP_CHECK(hipStreamSynchronize(s0));
        iters_max = std::max(iters_max, iter);
        {
            double mn_sum = 0.0;
            for (int lb = 0; lb < nb; ++lb) mn_sum += (double)bdesc[lb].m * bdesc[lb].n;
            rguess = std::min((double)rcap, std::max(4.0, 1.25 * (double)hused / std::max(mn_sum, 1.0)));
            p->faces_per_block[fpb_slot] = rguess;
        }
        if (p->opt.verbose) {
            size_t fb = 0, tb = 0;
            if (hipMemGetInfo(&fb, &tb) != hipSuccess) (void)hipGetLastError();
            std::fprintf(stderr, "gaca far field: batch of blocks %lld..%lld of %lld done, %d iterations, "
                         "%.1f ms since the start (%.1f ms waiting for the device, %.1f ms preparing and "
                         "%.1f ms enqueuing iterations, %.1f ms in %lld memory calls); factors %.2f GB, "
                         "fibres %.2f GB, face pool %.2f GB, free %.2f GB\n",
                         (long long)bt.first, (long long)bt.second, (long long)ntot, iter,
                         wall_ms_since(t_entry), ms_wait, ms_prep, ms_launch, (g_mem_ns.load() - mem_ns0) / 1e6,
                         (long long)(g_mem_calls.load() - mem_calls0),
                         (arena_used[0] + arena_used[1]) * es / 1e9, (fib_used[0] + fib_used[1]) * 16.0 / 1e9,
                         W.hpool.bytes / 1e9, fb / 1e9);
            std::fflush(stderr);
        }
        // give pool pages back between batches when memory is short (the arena needs them;
        // in-place pools regrow without copies).  Mapping fresh pages is slow (tens of ms per
        // GiB when the driver has to clear recently released memory), so pools stay mapped
        // while the free memory exceeds their size, and otherwise give back only the part
        // that leaves as much memory free as the face pool keeps
        if (bnext < ntot) {
            size_t fb = 0, tb = 0;
            if (hipMemGetInfo(&fb, &tb) != hipSuccess) {
                (void)hipGetLastError();
                fb = 0;
            }
            if (fb < W.hpool.bytes + W.fgpool.bytes) {
                if (W.fgpool.vmm) W.fgpool.shrink(0);
                if (W.hpool.vmm) W.hpool.shrink((fb + W.hpool.bytes) / 2);
            }
        }
    }
    // the pools hold no result; large ones are given back when memory is short
    {
        size_t held = W.hpool.bytes + W.fgpool.bytes + W.uw.bytes + W.part.bytes;
        size_t fb_end = 0, tb_end = 0;
        if (hipMemGetInfo(&fb_end, &tb_end) != hipSuccess) {
            (void)hipGetLastError();
            fb_end = 0;
        }
        // kept (mapped) for the problem's next build while they take at most half of the
        // device and leave a quarter of it free: remapping tens of GB costs seconds
        if (total_b > 0 && (held > total_b / 2 || fb_end < total_b / 4)) {
            W.hpool.release();
            W.fgpool.release();
            W.uw.release();
            W.part.release();
            W.rec_ws.release();
        }
    }
    GACA_HIP_CHECK(hipEventRecord(ev[EV_END], s0));
    GACA_HIP_CHECK(hipStreamWaitEvent(ctx->stream, ev[EV_END], 0));
    GACA_HIP_CHECK(hipEventSynchronize(ev[EV_END]));
    float span = 0.0f;
    GACA_HIP_CHECK(hipEventElapsedTime(&span, ev[EV_BEGIN], ev[EV_END]));
    const auto t_fin = std::chrono::steady_clock::now();
    if (nh > 1) {
        // joint tables -> each operator's own (rows w * nfar ... of the joint tables)
        for (int w = 0; w < nh; ++w) {
            gaca_hmatrix *hh = H[w];
            GACA_HIP_CHECK(hipMemcpyAsync(hh->d_meta.ptr, j_meta.as<FarMeta>() + w * nfar,
                                          nfar * sizeof(FarMeta), hipMemcpyDeviceToDevice, s0));
            GACA_HIP_CHECK(hipMemcpyAsync(hh->d_cmeta.ptr, j_cmeta.as<CrossMeta>() + w * nfar * rcap,
                                          nfar * rcap * sizeof(CrossMeta), hipMemcpyDeviceToDevice, s0));
            GACA_HIP_CHECK(hipMemcpyAsync(hh->d_cross_off.ptr, j_cross_off.as<int64_t>() + w * nfar * rcap,
                                          nfar * rcap * sizeof(int64_t), hipMemcpyDeviceToDevice, s0));
            GACA_HIP_CHECK(hipMemcpyAsync(hh->d_fib_off.ptr, j_fib_off.as<int64_t>() + w * nfar,
                                          nfar * sizeof(int64_t), hipMemcpyDeviceToDevice, s0));
        }
    }
    // result tables of every operator -> host through one pinned staging buffer, in stream
    // order after the joint-table split, with one synchronisation
    const size_t b_meta = nfar * sizeof(FarMeta), b_cmeta = (size_t)nfar * rcap * sizeof(CrossMeta),
                 b_coff = (size_t)nfar * rcap * sizeof(int64_t), b_foff = nfar * sizeof(int64_t);
    const size_t b_op = b_meta + b_cmeta + b_coff + b_foff;
    W.h_out.ensure(std::max<size_t>(b_op * nh, 1));
    for (int w = 0; w < nh; ++w) {
        gaca_hmatrix *hh = H[w];
        char *o = W.h_out.as<char>() + w * b_op;
        GACA_HIP_CHECK(hipMemcpyAsync(o, hh->d_meta.ptr, b_meta, hipMemcpyDeviceToHost, s0));
        GACA_HIP_CHECK(hipMemcpyAsync(o + b_meta, hh->d_cmeta.ptr, b_cmeta, hipMemcpyDeviceToHost, s0));
        GACA_HIP_CHECK(hipMemcpyAsync(o + b_meta + b_cmeta, hh->d_cross_off.ptr, b_coff,
                                      hipMemcpyDeviceToHost, s0));
        GACA_HIP_CHECK(hipMemcpyAsync(o + b_meta + b_cmeta + b_coff, hh->d_fib_off.ptr, b_foff,
                                      hipMemcpyDeviceToHost, s0));
    }
    GACA_HIP_CHECK(hipStreamSynchronize(s0));
    int wclk_khz = 0;
    if (hipDeviceGetAttribute(&wclk_khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess ||
        wclk_khz <= 0) {
        (void)hipGetLastError();
        wclk_khz = 100000;
    }
    for (int w = 0; w < nh; ++w) {
        gaca_hmatrix *hh = H[w];
        compact(ctx, hh->d_arena, arena_used[w] * es, s0);
        compact(ctx, hh->d_fib, fib_used[w] * sizeof(double2), s0);
        {
            const char *o = W.h_out.as<char>() + w * b_op;
            std::memcpy(hh->meta.data(), o, b_meta);
            std::memcpy(hh->cmeta.data(), o + b_meta, b_cmeta);
            std::memcpy(hh->cross_off.data(), o + b_meta + b_cmeta, b_coff);
            std::memcpy(hh->fib_off.data(), o + b_meta + b_cmeta + b_coff, b_foff);
        }
        // timings and work of the shared launches (identical in every operator of a joint build)
        gaca_stats &st = hh->st;
        st.joint_build = nh;
        st.ms_far_kernel = span;
        st.n_far_launches = n_launch;
        st.far_iters = iters_max;
        st.threads_large_used = p->opt.threads_large > 0 ? p->opt.threads_large : 512;
        st.threads_small_used = p->opt.threads_small;
        st.autotune_state = p->tune_state;
        st.far_kernel_evals = evals;
        st.far_flops = 0.0;
        for (int k = 0; k < 4; ++k) {
            st.ms_far_phase[k] = ms_phase[k];
            st.launches_phase[k] = launches_phase[k];
            st.far_flops_phase[k] = fl_phase[k];
            st.far_bytes_phase[k] = by_phase[k];
            st.far_flops += fl_phase[k];
        }
        for (int k = 0; k < 4; ++k) {
            st.ms_far_by_kind[k] = ms_kind[k];
            st.launches_by_kind[k] = launches_kind[k];
            st.far_flops_by_kind[k] = fl_kind[k];
            if (k < 3) {
                st.ms_far_large_path[k] = ms_path[k];
                st.launches_large_path[k] = launches_path[k];
                st.far_flops_large_path[k] = fl_path[k];
            }
        }
        int64_t tmax = 0;
        for (const auto &mt : hh->meta) tmax = std::max<int64_t>(tmax, mt.aca_ticks);
        st.ms_far_aca_block_max = (double)tmax / wclk_khz;
        st.ms_host_setup = ms_setup;
        st.arena_in_place = hh->d_arena.vmm ? 1 : 0;
    }
    for (gaca_hmatrix *hh : H) hh->st.ms_host_finish = wall_ms_since(t_fin);
}

static void fill_stats(gaca_hmatrix *h) {
    gaca_problem *p = h->p;
    gaca_stats &s = h->st;
    const int L = p->L;
    s.n_far = h->nfar;
    s.n_near = (int64_t)p->part.near.size();
    s.rank_min = h->nfar ? 1 << 30 : 0;
    s.rank_max = 0;
    double rsum = 0, frsum = 0, nfaces = 0;
    s.face_rank_max = 0;
    s.n_capped = 0;
    s.n_zero_blocks = 0;
    double far_elems = 0, fib_elems = 0;
    s.entries_face = s.entries_fibre = s.entries_face_kernel = 0;
    h->freq_hist.assign(L, 0);
    for (int64_t b = 0; b < h->nfar; ++b) {
        const FarMeta &mt = h->meta[b];
        const int m = (int)p->part.far[b][1], n = (int)p->part.far[b][3];
        s.rank_min = std::min(s.rank_min, mt.rank);
        s.rank_max = std::max(s.rank_max, mt.rank);
        rsum += mt.rank;
        if (mt.capped) s.n_capped++;
        if (mt.rank == 0) s.n_zero_blocks++;
        std::vector<char> used(L, 0);
        for (int c = 0; c < mt.rank; ++c) {
            const CrossMeta &cm = h->cmeta[b * h->rcap + c];
            s.face_rank_max = std::max(s.face_rank_max, cm.rho);
            frsum += cm.rho;
            nfaces += 1;
            far_elems += (double)cm.rho * (m + n);
            // entries read by the face ACA: rho rows of n and rho columns of m
            s.entries_face += (double)cm.rho * (m + n);
            used[cm.k] = 1;
        }
        // zero faces: every row of the face was tested
        s.entries_face += (double)mt.zero_faces * m * n;
        s.entries_face_kernel += (double)(mt.rank + mt.zero_faces) * m * n;
        s.entries_fibre += (double)mt.rank * L;
        fib_elems += (double)mt.rank * L;
        for (int k = 0; k < L; ++k) h->freq_hist[k] += used[k];
    }
    s.rank_mean = h->nfar ? rsum / h->nfar : 0.0;
    s.face_rank_mean = nfaces > 0 ? frsum / nfaces : 0.0;
    const double eb = h->prec == GACA_FP64 ? 16.0 : 8.0;
    s.bytes_far = (uint64_t)(far_elems * eb + fib_elems * 16.0);
    s.bytes_near = (uint64_t)((double)p->near_elems * eb);
    s.n_near_compressed = 0;
    s.near_rank_mean = 0.0;
    s.near_rank_max = 0;
    if (h->near_aca) {
        s.bytes_near = (uint64_t)((double)(h->near_faces_elems + h->near_dense_elems) * eb +
                                  (double)h->near_fib_elems * 16.0);
        double rs = 0.0;
        for (const auto &d : h->nblk_host)
            if (d.comp) {
                ++s.n_near_compressed;
                rs += d.crank;
                s.near_rank_max = std::max(s.near_rank_max, d.crank);
            }
        s.near_rank_mean = s.n_near_compressed ? rs / s.n_near_compressed : 0.0;
    }
    s.dense_bytes = (double)p->M * (double)p->M * L * eb;
    s.compression = (s.bytes_far + s.bytes_near) / std::max(1.0, s.dense_bytes);
    // with conjugate-pair frequencies the near kernels evaluate L_eval of the L frequencies
    // and write the others as conjugates
    s.entries_near = (double)p->near_elems * p->f.L_eval / std::max(1, p->f.L);
    s.entries_near_mirrored = (double)p->near_elems - s.entries_near;
}

// Builds the operators `kernels` (one, or the collocation single and double layer) of p:
// near fields on the context stream, far fields in one joint run.  Returns whether a rank
// cap was hit.
// 3D-ACA of the near blocks with dense faces (option near_aca), after the operator's build:
// chunks of blocks are compressed into scratch, the ranks read back, and each block's result
// packed into the operator's arenas (compressed: faces + fibres; otherwise: its dense
// [m][L][n] entries in a compact dense arena).  A block stays dense if its ACA hit the cap
// or rank (m n + L) >= m n L.  The dense near field of the build is then released.
static void near_compress(gaca_hmatrix *h) {
    gaca_problem *p = h->p;
    gaca_context *ctx = p->ctx;
    const hipStream_t st = ctx->stream;
    const int L = p->L;
    const bool fp32 = h->prec == GACA_MIXED;
    const size_t es = fp32 ? sizeof(float2) : sizeof(double2);
    const int64_t nb = (int64_t)p->nblocks.size();
    int mnmax = 1;
    for (const auto &b : p->nblocks) mnmax = std::max(mnmax, std::min(b.m * b.n, kNearAcaMaxMN));
    const int rc = std::max(1, std::min(L, 64));
    const double per = (double)rc * ((double)mnmax * es + L * 16.0) + 16.0;
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>(nb, (int64_t)((4.0 * (1 << 30)) / per)));
    DevBuf faces, fib, out, dst;
    faces.alloc(ctx, (size_t)chunk * rc * mnmax * es);
    fib.alloc(ctx, (size_t)chunk * rc * L * sizeof(double2));
    out.alloc(ctx, (size_t)chunk * sizeof(NearAcaOut));
    dst.alloc(ctx, (size_t)std::max<int64_t>(nb, 1) * sizeof(NearBlockDev));
    std::vector<NearAcaOut> res((size_t)chunk);
    h->nblk_host = p->nblocks;
    int64_t fu = 0, gu = 0, du = 0;   // used elements of the face, fibre, dense arenas
    NearAcaArgs q{};
    q.blocks = p->d_nblocks.as<NearBlockDev>();
    q.L = L;
    q.rc = rc;
    q.mnmax = mnmax;
    q.eps = p->opt.eps3d;
    q.tie = fp32 ? std::max(p->opt.tie, 1e-4) : p->opt.tie;
    q.delta = fp32 ? std::max(p->opt.delta_zero, 1e-6) : p->opt.delta_zero;
    q.fib = fib.as<double2>();
    q.out = out.as<NearAcaOut>();
    for (int64_t b0 = 0; b0 < nb; b0 += chunk) {
        const int n = (int)std::min<int64_t>(chunk, nb - b0);
        q.b0 = b0;
        launch_near_aca(q, n, h->d_near.ptr, faces.ptr, fp32 ? 1 : 0, st);
        GACA_HIP_CHECK(hipGetLastError());
        GACA_HIP_CHECK(hipMemcpyAsync(res.data(), out.ptr, n * sizeof(NearAcaOut), hipMemcpyDeviceToHost, st));
        GACA_HIP_CHECK(hipStreamSynchronize(st));
        const int64_t fu0 = fu, gu0 = gu, du0 = du;
        for (int t = 0; t < n; ++t) {
            NearBlockDev &d = h->nblk_host[b0 + t];
            const int64_t mn = (int64_t)d.m * d.n;
            const NearAcaOut &r = res[t];
            if (!r.capped && mn <= kNearAcaMaxMN && (int64_t)r.rank * (mn + L) < mn * L) {
                d.comp = 1;
                d.crank = r.rank;
                d.off = fu;
                d.foff = gu;
                fu += (int64_t)r.rank * mn;
                gu += (int64_t)r.rank * L;
            } else {
                d.comp = 0;
                d.crank = 0;
                d.off = du;
                d.foff = 0;
                du += mn * L;
            }
        }
        grow_keep(ctx, h->n_faces, (size_t)std::max<int64_t>(fu, 1) * es, (size_t)fu0 * es, st);
        grow_keep(ctx, h->n_fib, (size_t)std::max<int64_t>(gu, 1) * sizeof(double2), (size_t)gu0 * sizeof(double2), st);
        grow_keep(ctx, h->n_dense, (size_t)std::max<int64_t>(du, 1) * es, (size_t)du0 * es, st);
        GACA_HIP_CHECK(hipMemcpyAsync(dst.as<NearBlockDev>() + b0, h->nblk_host.data() + b0,
                                      n * sizeof(NearBlockDev), hipMemcpyHostToDevice, st));
        launch_near_aca_pack(q, n, h->d_near.ptr, faces.ptr, dst.as<NearBlockDev>(), h->n_faces.ptr,
                             h->n_fib.as<double2>(), h->n_dense.ptr, fp32 ? 1 : 0, st);
        GACA_HIP_CHECK(hipGetLastError());
        GACA_HIP_CHECK(hipStreamSynchronize(st));   // the host table of the chunk is reused
    }
    h->d_nblk_own.swap(dst);
    h->near_faces_elems = fu;
    h->near_fib_elems = gu;
    h->near_dense_elems = du;
    h->near_aca = true;
    h->d_near.release();
}

static void prepare_leaves(gaca_hmatrix *h);

static bool build_ops(gaca_problem *p, const std::vector<gaca_kernel> &kernels,
                      std::vector<std::unique_ptr<gaca_hmatrix>> &out) {
    REQUIRE(!p->synthetic, "build needs a mesh problem");
    REQUIRE(p->opt.precision == GACA_FP64 || p->opt.precision == GACA_MIXED, "bad precision");
    for (gaca_kernel kernel : kernels) {
        REQUIRE(kernel == GACA_SLP || kernel == GACA_DLP || kernel == GACA_HYP || kernel == GACA_ADLP,
                "bad kernel");
        if (p->scheme == GACA_GALERKIN_P0 && kernel != GACA_SLP)
            throw Error{GACA_ERR_UNSUPPORTED, "Galerkin is available for the single layer only"};
        if (p->scheme == GACA_COLLOCATION_P1 && kernel != GACA_DLP)
            throw Error{GACA_ERR_UNSUPPORTED, "the P1 scheme has the double layer only"};
        if ((p->scheme == GACA_GALERKIN_P1) != (kernel == GACA_HYP || kernel == GACA_ADLP))
            throw Error{GACA_ERR_UNSUPPORTED,
                        "the hypersingular operator and the adjoint double layer belong to the Galerkin P1 scheme"};
    }
    gaca_context *ctx = p->ctx;
    GACA_HIP_CHECK(hipSetDevice(ctx->device));
    const hipStream_t st = ctx->stream;
    const bool mixed = p->opt.precision == GACA_MIXED;
    const int nh = (int)kernels.size();
    std::vector<gaca_hmatrix *> H;
    out.clear();
    for (gaca_kernel kernel : kernels) {
        auto h = std::make_unique<gaca_hmatrix>();
        h->p = p;
        p->nops += 1;
        h->kernel = p->kid(kernel);
        h->prec = p->opt.precision;
        h->rcap = std::max(1, std::min({p->L, p->opt.max_rank3d > 0 ? p->opt.max_rank3d : p->L, 256}));
        // near field: FP64 quadrature, stored FP64 or (mixed) FP32 (every entry is written)
        const size_t nbytes = std::max<int64_t>(1, p->near_elems) * (mixed ? sizeof(float2) : sizeof(double2));
        {
            std::lock_guard<std::mutex> lk(p->spare_mu);
            DevBuf &sp = p->near_spare[h->kernel & 1];
            if (sp.ptr && sp.bytes == nbytes) h->d_near.swap(sp);
        }
        if (!h->d_near.ptr) h->d_near.alloc(ctx, nbytes);
        H.push_back(h.get());
        out.push_back(std::move(h));
    }
    // events: begin, then per operator near start / near end, then end
    std::vector<hipEvent_t> ev(2 + 2 * nh);
    for (auto &e : ev) GACA_HIP_CHECK(hipEventCreate(&e));
    struct EvGuard {
        std::vector<hipEvent_t> &e;
        ~EvGuard() {
            for (auto x : e) (void)hipEventDestroy(x);
        }
    } ev_guard{ev};
    GACA_HIP_CHECK(hipEventRecord(ev[0], st));
    auto near_work = [&] {
        for (int w = 0; w < nh; ++w) {
            gaca_hmatrix *h = H[w];
            GACA_HIP_CHECK(hipEventRecord(ev[1 + 2 * w], st));
            double2 *n64 = mixed ? nullptr : h->d_near.as<double2>();
            float2 *n32 = mixed ? h->d_near.as<float2>() : nullptr;
            if (p->scheme == GACA_COLLOCATION_P1)
                launch_near_p1(p->g, p->q, p->f, p->d_pairs[0].as<NearPair>(), p->npairs[0],
                               p->d_nblocks.as<NearBlockDev>(), n64, st);
            if (p->scheme == GACA_GALERKIN_P1)
                launch_near_gp1(kernels[w] == GACA_HYP ? 0 : 1, p->g, p->q, p->f, p->d_pairs[0].as<NearPair>(),
                                p->npairs[0], p->d_nblocks.as<NearBlockDev>(), n64, st);
            for (int t = 0; t < kNumTiers && !p->p1(); ++t) {
                if (p->scheme == GACA_GALERKIN_P0)
                    launch_near_galerkin(t, p->g, p->q, p->f, p->d_pairs[t].as<NearPair>(),
                                         p->npairs[t], p->d_nblocks.as<NearBlockDev>(), n64, n32, st);
                else if (t < 4)
                    launch_near(kernels[w], t, p->g, p->q, p->f, p->d_pairs[t].as<NearPair>(),
                                p->npairs[t], p->d_nblocks.as<NearBlockDev>(), n64, n32, st);
            }
            GACA_HIP_CHECK(hipGetLastError());
            GACA_HIP_CHECK(hipEventRecord(ev[2 + 2 * w], st));
        }
    };
    run_far(H, nullptr, near_work);
    GACA_HIP_CHECK(hipEventRecord(ev[1 + 2 * nh], st));
    GACA_HIP_CHECK(hipEventSynchronize(ev[1 + 2 * nh]));
    float ms_total = 0;
    GACA_HIP_CHECK(hipEventElapsedTime(&ms_total, ev[0], ev[1 + 2 * nh]));
    bool capped = false;
    for (int w = 0; w < nh; ++w) {
        gaca_hmatrix *h = H[w];
        float ms_near = 0;
        GACA_HIP_CHECK(hipEventElapsedTime(&ms_near, ev[1 + 2 * w], ev[2 + 2 * w]));
        fill_stats(h);
        h->st.ms_near = ms_near;
        h->st.ms_near_kernel = ms_near;
        const double le = p->f.L_eval;
        const double ng2 = (double)p->opt.n_galerkin * p->opt.n_galerkin;
        const double nm2 = (double)p->opt.quad_mid * p->opt.quad_mid;
        const double nn2 = (double)p->opt.quad_near * p->opt.quad_near;
        const double ns = p->opt.n_touch;
        double qp[kNumTiers] = {6.0, nm2, nn2, kernels[w] == 0 ? 3.0 * p->opt.n_duffy * p->opt.n_duffy : 0.0,
                                0.0, 0.0};
        if (p->scheme == GACA_GALERKIN_P0) {
            // touching pairs: 5 n^2 (edge) and 2 n^3 (vertex) evaluations of the exact radial
            // integrals per frequency
            const double g6[kNumTiers] = {36.0, nm2 * nm2, 3.0 * ng2 * ng2, 5.0 * ns * ns,
                                          2.0 * ns * ns * ns, 6.0 * kGalerkinNTheta};
            for (int t = 0; t < kNumTiers; ++t) qp[t] = g6[t];
        }
        double evn = 0.0;
        for (int t = 0; t < kNumTiers; ++t) evn += (double)p->npairs[t] * le * qp[t];
        if (p->p1()) evn = p->p1_near_points * le;
        h->st.near_kernel_evals = evn;
        h->st.ms_far = h->st.ms_far_kernel;
        h->st.ms_total = ms_total;
        capped = capped || h->st.n_capped > 0;
    }
    if (p->opt.near_aca)
        for (int w = 0; w < nh; ++w) {
            const auto t0 = std::chrono::steady_clock::now();
            near_compress(H[w]);
            fill_stats(H[w]);
            H[w]->st.ms_near_aca =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
    // leaf tables of the apply (per problem, once): built here so that no apply allocates them
    prepare_leaves(out[0].get());
    return capped;
}

// ---------------------------------------------------------------------------------------
// Autotuner of the face-ACA workgroup sizes (threads_large, threads_small): with an
// autotune_cache file and threads_large = 0, the first build of a problem looks its
// workload up in the file; if absent, it builds the operators once per candidate, keeps the
// one whose face-ACA phase (device time of the aca launches) was shortest, returns that
// build and appends the choice to the file.  Later builds of the problem reuse the choice.
}  // extern "C"

namespace {
const int kTuneCand[][2] = {{512, 128}, {1024, 128}, {512, 64}, {256, 128}};

std::string tune_key(const gaca_problem *p, const std::vector<gaca_kernel> &kernels) {
    char buf[512];
    std::string ops;
    for (gaca_kernel k : kernels) ops += k == GACA_SLP ? "s" : "d";
    std::snprintf(buf, sizeof(buf), "v1|M=%lld|L=%d|scheme=%d|ops=%s|prec=%d|leaf=%d|eta=%.6g|eps=%.6g|"
                  "epsaca=%.6g|nfar=%lld|cu=%d",
                  (long long)p->M, p->L, (int)p->scheme, ops.c_str(), (int)p->opt.precision,
                  p->opt.leaf_size, p->opt.eta, p->opt.eps3d, p->opt.eps_aca,
                  (long long)p->part.far.size(), p->ctx->n_cu);
    return buf;
}

bool tune_lookup(const std::string &path, const std::string &key, int &tl, int &ts) {
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return false;
    char line[1024];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char k[900];
        int a = 0, b = 0;
        if (std::sscanf(line, "%899s %d %d", k, &a, &b) == 3 && key == k && (a == 256 || a == 512 || a == 1024) &&
            (b == 64 || b == 128)) {
            tl = a;
            ts = b;
            found = true;   // the last entry for the key wins
        }
    }
    std::fclose(f);
    return found;
}
}  // namespace

extern "C" {

static bool build_ops(gaca_problem *p, const std::vector<gaca_kernel> &kernels,
                      std::vector<std::unique_ptr<gaca_hmatrix>> &out);

static bool build_tuned(gaca_problem *p, const std::vector<gaca_kernel> &kernels,
                        std::vector<std::unique_ptr<gaca_hmatrix>> &out) {
    const int tl0 = p->opt.threads_large, ts0 = p->opt.threads_small;
    if (!p->opt.autotune_cache || tl0 != 0) return build_ops(p, kernels, out);
    struct Restore {
        gaca_problem *p;
        int tl, ts;
        ~Restore() {
            p->opt.threads_large = tl;
            p->opt.threads_small = ts;
        }
    } restore{p, tl0, ts0};
    if (!p->tuned_tl) {
        int tl = 0, ts = 0;
        if (tune_lookup(p->autotune_path, tune_key(p, kernels), tl, ts)) {
            p->tuned_tl = tl;
            p->tuned_ts = ts;
            p->tune_state = 2;
        }
    }
    if (p->tuned_tl) {
        p->opt.threads_large = p->tuned_tl;
        p->opt.threads_small = p->tuned_ts;
        return build_ops(p, kernels, out);
    }
    double best = 1e300;
    bool best_capped = false;
    std::vector<std::unique_ptr<gaca_hmatrix>> best_hs;
    for (const auto &c : kTuneCand) {
        p->opt.threads_large = c[0];
        p->opt.threads_small = c[1];
        std::vector<std::unique_ptr<gaca_hmatrix>> hs;
        const bool capped = build_ops(p, kernels, hs);
        const double t = hs[0]->st.ms_far_phase[1];
        if (t < best) {
            for (auto &h : best_hs) gaca_hmatrix_destroy(h.release());
            best_hs = std::move(hs);
            best = t;
            best_capped = capped;
            p->tuned_tl = c[0];
            p->tuned_ts = c[1];
        } else {
            for (auto &h : hs) gaca_hmatrix_destroy(h.release());
        }
    }
    p->tune_state = 1;
    for (auto &h : best_hs) h->st.autotune_state = 1;
    if (FILE *f = std::fopen(p->autotune_path.c_str(), "a")) {
        std::fprintf(f, "%s %d %d\n", tune_key(p, kernels).c_str(), p->tuned_tl, p->tuned_ts);
        std::fclose(f);
    }
    out = std::move(best_hs);
    return best_capped;
}

gaca_status gaca_build(gaca_problem *p, gaca_kernel kernel, gaca_hmatrix **out) {
    bool capped = false;
    gaca_status rc = guarded([&] {
        REQUIRE(p && out, "null argument");
        std::vector<std::unique_ptr<gaca_hmatrix>> hs;
        capped = build_tuned(p, {kernel}, hs);
        *out = hs[0].release();
    });
    if (rc == GACA_OK && capped) {
        set_error("rank cap hit in at least one block");
        return GACA_ERR_NOT_CONVERGED;
    }
    return rc;
}

gaca_status gaca_build_both(gaca_problem *p, gaca_hmatrix **slp_out, gaca_hmatrix **dlp_out) {
    bool capped = false;
    gaca_status rc = guarded([&] {
        REQUIRE(p && slp_out && dlp_out, "null argument");
        if (p->scheme == GACA_GALERKIN_P0)
            throw Error{GACA_ERR_UNSUPPORTED, "Galerkin is available for the single layer only"};
        if (p->p1())
            throw Error{GACA_ERR_UNSUPPORTED, "joint builds are for the P0 collocation operators"};
        std::vector<std::unique_ptr<gaca_hmatrix>> hs;
        capped = build_tuned(p, {GACA_SLP, GACA_DLP}, hs);
        *slp_out = hs[0].release();
        *dlp_out = hs[1].release();
    });
    if (rc == GACA_OK && capped) {
        set_error("rank cap hit in at least one block");
        return GACA_ERR_NOT_CONVERGED;
    }
    return rc;
}

gaca_status gaca_hmatrix_destroy(gaca_hmatrix *h) {
    if (h && h->p && !h->owned_problem) {
        // keep mapped arenas of moderate size for the problem's next build
        gaca_problem *p = h->p;
        size_t fb = 0, tb = 0;
        if (hipMemGetInfo(&fb, &tb) != hipSuccess) {
            (void)hipGetLastError();
            tb = 0;
        }
        std::lock_guard<std::mutex> lk(p->spare_mu);
        bool synced = false;
        // into the slot of the operator's kind only: a build takes one arena of its kind, so
        // a second spare of that kind would stay mapped and idle, taking memory that the next
        // build's far-field batch could use
        auto donate = [&](GrowBuf &src, GrowBuf *spare) {
            if (!src.vmm || !src.ptr || src.bytes > tb / 8) return;
            const int k = h->kernel & 1;
            if (spare[k].ptr) return;
            if (!synced) {
                (void)hipDeviceSynchronize();   // no kernel may still use the arena
                synced = true;
            }
            spare[k].swap(src);
        };
        donate(h->d_arena, p->spare_arena);
        donate(h->d_fib, p->spare_fib);
        // near field of the same size as the next build's (kept up to an eighth of the memory)
        {
            DevBuf &sp = p->near_spare[h->kernel & 1];
            if (h->d_near.ptr && h->d_near.bytes <= tb / 8 && !sp.ptr) {
                if (!synced) {
                    (void)hipDeviceSynchronize();
                    synced = true;
                }
                sp.swap(h->d_near);
            }
        }
        // far-field result tables (device and host) for the next build of the same size
        {
            const int k = h->kernel & 1;
            DevBuf *tabs[5] = {&h->d_meta, &h->d_cmeta, &h->d_cross_off, &h->d_fib_off, &h->d_far4};
            for (int t = 0; t < 5; ++t) {
                if (!tabs[t]->ptr || p->tab_spare[k][t].ptr) continue;
                if (!synced) {
                    (void)hipDeviceSynchronize();   // no kernel may still read the table
                    synced = true;
                }
                p->tab_spare[k][t].swap(*tabs[t]);
            }
            if (p->cmeta_spare[k].empty()) {
                p->meta_spare[k].swap(h->meta);
                p->cmeta_spare[k].swap(h->cmeta);
                p->coff_spare[k].swap(h->cross_off);
                p->foff_spare[k].swap(h->fib_off);
            }
        }
        // VALU apply workspace: kept when no larger buffer of its kind is kept already
        DevBuf *ws[5] = {&h->d_yb, &h->d_z, &h->d_t, &h->d_xp, &h->d_yp};
        for (int k = 0; k < 5; ++k) {
            if (!ws[k]->ptr || ws[k]->bytes > tb / 16 || p->ws_spare[k].bytes >= ws[k]->bytes) continue;
            if (!synced) {
                (void)hipDeviceSynchronize();   // no kernel may still use the buffer
                synced = true;
            }
            p->ws_spare[k].swap(*ws[k]);
        }
    }
    delete h;
    return GACA_OK;
}

gaca_status gaca_hmatrix_stats(const gaca_hmatrix *h, gaca_stats *st) {
    return guarded([&] {
        REQUIRE(h && st, "null argument");
        *st = h->st;
    });
}

gaca_status gaca_hmatrix_freq_hist(const gaca_hmatrix *h, int64_t *hist) {
    return guarded([&] {
        REQUIRE(h && hist, "null argument");
        std::copy(h->freq_hist.begin(), h->freq_hist.end(), hist);
    });
}

gaca_status gaca_hmatrix_block_info(const gaca_hmatrix *h, int64_t idx, int64_t *info) {
    return guarded([&] {
        REQUIRE(h && info, "null argument");
        REQUIRE(idx >= 0 && idx < h->nfar, "block index out of range");
        const auto &blk = h->p->part.far[idx];
        const FarMeta &mt = h->meta[idx];
        info[0] = blk[0];
        info[1] = blk[1];
        info[2] = blk[2];
        info[3] = blk[3];
        info[4] = mt.rank;
        info[5] = mt.sum_rho;
        info[6] = mt.capped;
        info[7] = mt.zero_faces;
        info[8] = mt.aca_ticks;
    });
}

gaca_status gaca_hmatrix_block_export(const gaca_hmatrix *h, int64_t idx, int32_t *ks,
                                      int32_t *pi, int32_t *pj, int32_t *rho, double *U,
                                      double *W, double *F) {
    return guarded([&] {
        REQUIRE(h, "null handle");
        REQUIRE(idx >= 0 && idx < h->nfar, "block index out of range");
        const auto &blk = h->p->part.far[idx];
        const int64_t m = blk[1], n = blk[3];
        const int L = h->p->L;
        const FarMeta &mt = h->meta[idx];
        int64_t uo = 0, wo = 0;
        for (int c = 0; c < mt.rank; ++c) {
            const CrossMeta &cm = h->cmeta[idx * h->rcap + c];
            const int64_t off = h->cross_off[idx * h->rcap + c];
            if (ks) ks[c] = cm.k;
            if (pi) pi[c] = cm.pi;
            if (pj) pj[c] = cm.pj;
            if (rho) rho[c] = cm.rho;
            if (off < 0) throw Error{GACA_ERR_STATE, "factors missing (arena overflow)"};
            // factors are double2 (FP64) or float2 (mixed); exported widened to C128
            auto fetch = [&](double *dst, int64_t eoff, int64_t cnt) {
                if (h->prec == GACA_MIXED) {
                    std::vector<float> tmp(2 * cnt);
                    GACA_HIP_CHECK(hipMemcpy(tmp.data(), h->d_arena.as<float2>() + eoff,
                                             cnt * sizeof(float2), hipMemcpyDeviceToHost));
                    for (int64_t t = 0; t < 2 * cnt; ++t) dst[t] = tmp[t];
                } else {
                    GACA_HIP_CHECK(hipMemcpy(dst, h->d_arena.as<double2>() + eoff,
                                             cnt * sizeof(double2), hipMemcpyDeviceToHost));
                }
            };
            if (U) fetch(U + 2 * uo, off, (int64_t)cm.rho * m);
            if (W) fetch(W + 2 * wo, off + (int64_t)cm.rho * m, (int64_t)cm.rho * n);
            uo += (int64_t)cm.rho * m;
            wo += (int64_t)cm.rho * n;
        }
        if (F && mt.rank > 0) {
            REQUIRE(h->fib_off[idx] >= 0, "fibres missing");
            GACA_HIP_CHECK(hipMemcpy(F, h->d_fib.as<double2>() + h->fib_off[idx],
                                     (size_t)mt.rank * L * sizeof(double2), hipMemcpyDeviceToHost));
        }
    });
}

gaca_status gaca_hmatrix_near_export(const gaca_hmatrix *h, int64_t idx, double *out) {
    return guarded([&] {
        REQUIRE(h && out, "null argument");
        REQUIRE(idx >= 0 && idx < (int64_t)h->p->nblocks.size(), "near block index out of range");
        const NearBlockDev &nb = h->near_aca ? h->nblk_host[idx] : h->p->nblocks[idx];
        const size_t cnt = (size_t)nb.m * nb.n * h->p->L;
        if (h->near_aca) {
            gaca_context *ctx = h->p->ctx;
            DevBuf tmp;
            tmp.alloc(ctx, cnt * sizeof(double2));
            const bool fp32 = h->prec == GACA_MIXED;
            if (nb.comp) {
                launch_near_aca_expand(nb, h->p->L, h->n_faces.ptr, h->n_fib.as<double2>(),
                                       tmp.as<double2>(), fp32 ? 1 : 0, ctx->stream);
                GACA_HIP_CHECK(hipGetLastError());
                GACA_HIP_CHECK(hipStreamSynchronize(ctx->stream));
                GACA_HIP_CHECK(hipMemcpy(out, tmp.ptr, cnt * sizeof(double2), hipMemcpyDeviceToHost));
            } else if (!fp32) {
                GACA_HIP_CHECK(hipMemcpy(out, h->n_dense.as<double2>() + nb.off, cnt * sizeof(double2),
                                         hipMemcpyDeviceToHost));
            } else {
                std::vector<float> t32(2 * cnt);
                GACA_HIP_CHECK(hipMemcpy(t32.data(), h->n_dense.as<float2>() + nb.off, cnt * sizeof(float2),
                                         hipMemcpyDeviceToHost));
                for (size_t t = 0; t < 2 * cnt; ++t) out[t] = t32[t];
            }
            return;
        }
        if (h->prec == GACA_FP64) {
            GACA_HIP_CHECK(hipMemcpy(out, h->d_near.as<double2>() + nb.off, cnt * sizeof(double2),
                                     hipMemcpyDeviceToHost));
        } else {
            std::vector<float> tmp(2 * cnt);
            GACA_HIP_CHECK(hipMemcpy(tmp.data(), h->d_near.as<float2>() + nb.off, cnt * sizeof(float2),
                                     hipMemcpyDeviceToHost));
            for (size_t t = 0; t < 2 * cnt; ++t) out[t] = tmp[t];
        }
    });
}

gaca_status gaca_hmatrix_near_ranks(const gaca_hmatrix *h, int32_t *ranks) {
    return guarded([&] {
        REQUIRE(h && ranks, "null argument");
        const size_t nb = h->p->nblocks.size();
        for (size_t b = 0; b < nb; ++b)
            ranks[b] = h->near_aca && h->nblk_host[b].comp ? h->nblk_host[b].crank : -1;
    });
}

// ---------------------------------------------------------------------------------------
static void prepare_leaves(gaca_hmatrix *h) {
    gaca_problem *p = h->p;
    std::lock_guard<std::mutex> lk(p->leaf_mu);
    if (p->leaf_ready) return;
    gaca_context *ctx = p->ctx;
    const size_t nleaf = p->leaf_r0.size();
    std::vector<std::vector<int32_t>> lf(nleaf), ln(nleaf);
    auto leaves_in = [&](int64_t r0, int64_t m, auto &&fn) {
        auto it = std::lower_bound(p->leaf_r0.begin(), p->leaf_r0.end(), (int32_t)r0);
        for (size_t k = it - p->leaf_r0.begin(); k < nleaf && p->leaf_r0[k] < r0 + m; ++k) fn(k);
    };
    for (size_t b = 0; b < p->part.far.size(); ++b)
        leaves_in(p->part.far[b][0], p->part.far[b][1], [&](size_t k) { lf[k].push_back((int32_t)b); });
    for (size_t b = 0; b < p->part.near.size(); ++b)
        leaves_in(p->part.near[b][0], p->part.near[b][1], [&](size_t k) { ln[k].push_back((int32_t)b); });
    std::vector<int32_t> fp{0}, fi, np{0}, ni;
    for (size_t k = 0; k < nleaf; ++k) {
        fi.insert(fi.end(), lf[k].begin(), lf[k].end());
        fp.push_back((int32_t)fi.size());
        ni.insert(ni.end(), ln[k].begin(), ln[k].end());
        np.push_back((int32_t)ni.size());
    }
    p->d_leaf_r0.upload(ctx, p->leaf_r0);
    p->d_leaf_m.upload(ctx, p->leaf_m);
    p->d_lfp.upload(ctx, fp);
    p->d_lfi.upload(ctx, fi);
    p->d_lnp.upload(ctx, np);
    p->d_lni.upload(ctx, ni);
    p->leaf_ready = true;
}

// Workspace of the VALU apply (tree-order copies of X and Y, z, t and per-block y).
static void alloc_apply_workspace(gaca_hmatrix *h, gaca_apply_mode mode, int32_t nrhs, gaca_dtype dtype) {
    gaca_problem *p = h->p;
    gaca_context *ctx = p->ctx;
    const int L = p->L;
    const int64_t M = p->M;
    const size_t xs = dtype == GACA_C64 ? sizeof(float2) : sizeof(double2);
    {
            std::vector<int64_t> zoff(std::max<int64_t>(h->nfar, 1)), toff(std::max<int64_t>(h->nfar, 1)),
                yoff(std::max<int64_t>(h->nfar, 1));
            // crosses per T group: up to kApplyCB while the T workspace stays within 2 GiB
            int64_t nsum = 0;
            for (int64_t b = 0; b < h->nfar; ++b) nsum += p->part.far[b][3];
            const double t_one = (double)nsum * nrhs * xs;
            const int cb = mode == GACA_APPLY_SUM
                               ? (int)std::max(1.0, std::min((double)kApplyCB, std::floor(2147483648.0 / std::max(t_one, 1.0))))
                               : 1;
            int64_t zacc = 0, tacc = 0, yacc = 0;
            for (int64_t b = 0; b < h->nfar; ++b) {
                zoff[b] = zacc;
                toff[b] = tacc;
                yoff[b] = yacc;
                yacc += p->part.far[b][1] * (int64_t)nrhs;
                const int64_t sr = h->meta[b].sum_rho;
                zacc += mode == GACA_APPLY_SUM ? sr * nrhs : sr * (int64_t)L * nrhs;
                tacc += mode == GACA_APPLY_SUM ? std::min<int64_t>(h->meta[b].rank, cb) *
                                                     p->part.far[b][3] * (int64_t)nrhs
                                               : 0;
            }
            h->d_zoff.upload(ctx, zoff);
            h->d_toff.upload(ctx, toff);
            h->d_yoff.upload(ctx, yoff);
            // a buffer handed back by an operator of the same problem serves when it is large
            // enough (every byte of the workspace is written before it is read)
            auto take = [&](DevBuf &dst, int slot, size_t need) {
                if (dst.ptr && dst.bytes >= need) return;
                dst.release();
                {
                    std::lock_guard<std::mutex> lk(p->spare_mu);
                    DevBuf &sp = p->ws_spare[slot];
                    if (sp.ptr && sp.bytes >= need) {
                        dst.swap(sp);
                        return;
                    }
                }
                dst.alloc(ctx, need);
            };
            const int nl = mode == GACA_APPLY_SUM ? 1 : L;
            take(h->d_yb, 0, (size_t)std::max<int64_t>(yacc, 1) * xs);
            take(h->d_z, 1, (size_t)std::max<int64_t>(zacc, 1) * xs);
            take(h->d_t, 2, (size_t)std::max<int64_t>(tacc, 1) * xs);
            take(h->d_xp, 3, (size_t)L * M * nrhs * xs);
            take(h->d_yp, 4, (size_t)nl * M * nrhs * xs);
            if (h->near_aca) {
                // T_l of each compressed near block: [crank][n][nrhs]
                std::vector<int64_t> tnoff(std::max<size_t>(h->nblk_host.size(), 1), 0);
                int64_t tn = 0;
                for (size_t b = 0; b < h->nblk_host.size(); ++b) {
                    tnoff[b] = tn;
                    const NearBlockDev &d = h->nblk_host[b];
                    if (d.comp && mode == GACA_APPLY_SUM) tn += (int64_t)d.crank * d.n * nrhs;
                }
                h->d_tnoff.upload(ctx, tnoff);
                h->d_tn.release();
                h->d_tn.alloc(ctx, (size_t)std::max<int64_t>(tn, 1) * xs);
            }
            h->ws_nrhs = nrhs;
            h->ws_mode = (int)mode;
            h->ws_dtype = (int)dtype;
            h->ws_cb = cb;
        }
}

// The matrix-core apply stages the U rows of one far block by their sum of face ranks and
// the X rows of one near block by its columns.
static bool mfma_supported(const gaca_hmatrix *h) {
    if (h->near_aca) return false;   // compressed near blocks: the VALU apply
    for (int64_t b = 0; b < h->nfar; ++b)
        if (h->meta[b].sum_rho > kMfmaMaxSumRho) return false;
    for (const auto &nb : h->p->nblocks)
        if (nb.n > kMfmaMaxNearCols) return false;
    return true;
}

// SUM mode on the matrix cores: right-hand sides in chunks of up to 64 columns; per chunk
// the far blocks in batches whose T fits the workspace, then one pass over the leaves.
static void apply_mfma(gaca_hmatrix *h, const ApplyDev &a, int32_t nrhs, const float2 *X,
                       float2 *Y, hipStream_t st) {
    gaca_problem *p = h->p;
    gaca_context *ctx = p->ctx;
    const int64_t nfar = h->nfar;
    std::vector<int32_t> sum_rho(std::max<int64_t>(nfar, 1), 0);
    int64_t rho_tot = 0;
    for (int64_t b = 0; b < nfar; ++b) {
        sum_rho[b] = h->meta[b].sum_rho;
        rho_tot += sum_rho[b];
    }
    // right-hand sides per chunk: a power of two up to 64 (the kernels split column indices
    // with shifts; columns past the last right-hand side are zero), halved while Z (sum of
    // face ranks x chunk) would exceed 40 % of the free memory
    int nrc_max = 64;
    while (nrc_max > 1 && nrc_max / 2 >= nrhs) nrc_max /= 2;
    {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && rho_tot > 0) {
            free_b += h->d_mz.bytes;   // this operator's Z workspace of an earlier call is reused
            while (nrc_max > 1 && (double)rho_tot * nrc_max * sizeof(float2) > 0.4 * (double)free_b)
                nrc_max /= 2;
        } else {
            (void)hipGetLastError();
        }
    }
    h->d_msumrho.upload(ctx, sum_rho);
    ensure(ctx, h->d_mz, (size_t)std::max<int64_t>(rho_tot * nrc_max, 1) * sizeof(float2));
    int max_leaf = 1;
    for (int32_t m : p->leaf_m) max_leaf = std::max(max_leaf, m);
    const int row_tiles = (max_leaf + 31) / 32;
    // algorithmic work of the whole apply (complex multiply-add = 8 flops): far T = F X
    // (r L n per rhs), far Z = W T (sum_rho n), leaf (near m n L + far U Z: sum_rho m)
    {
        const int L = p->L;
        double mt = 0.0, mz = 0.0, ml = (double)p->near_elems;
        for (int64_t b = 0; b < nfar; ++b) {
            const double m = (double)p->part.far[b][1], n = (double)p->part.far[b][3];
            mt += (double)h->meta[b].rank * L * n;
            mz += (double)sum_rho[b] * n;
            ml += (double)sum_rho[b] * m;
        }
        h->st.apply_flops_part[0] = 8.0 * mt * nrhs;
        h->st.apply_flops_part[1] = 8.0 * mz * nrhs;
        h->st.apply_flops_part[2] = 8.0 * ml * nrhs;
        h->st.apply_flops = 8.0 * (mt + mz + ml) * nrhs;
        h->st.apply_operator_bytes = (double)(h->st.bytes_far + h->st.bytes_near);
    }
    hipEvent_t ev0, ev1, ep[4];
    GACA_HIP_CHECK(hipEventCreate(&ev0));
    GACA_HIP_CHECK(hipEventCreate(&ev1));
    for (auto &e : ep) GACA_HIP_CHECK(hipEventCreate(&e));
    double ms_part[3] = {0, 0, 0};
    auto part_ms = [&](int x, int y) {
        float ms = 0.0f;
        GACA_HIP_CHECK(hipEventElapsedTime(&ms, ep[x], ep[y]));
        return (double)ms;
    };
    GACA_HIP_CHECK(hipEventRecord(ev0, st));
    const size_t t_budget = (size_t)1 << 31;   // bytes of T per far batch
    // far blocks grouped by column cluster (tree-order start and size), in first-seen order
    std::vector<std::vector<int64_t>> groups;
    {
        std::map<std::pair<int64_t, int64_t>, size_t> gid;
        for (int64_t b = 0; b < nfar; ++b) {
            const auto key = std::make_pair(p->part.far[b][2], p->part.far[b][3]);
            auto it = gid.find(key);
            if (it == gid.end()) {
                gid.emplace(key, groups.size());
                groups.push_back({b});
            } else {
                groups[it->second].push_back(b);
            }
        }
    }
    for (int c0 = 0; c0 < nrhs; c0 += nrc_max) {
        const int ncur = std::min(nrc_max, nrhs - c0);
        int nrc = 1;
        while (nrc < ncur) nrc *= 2;
        int lg = 0;
        while ((1 << lg) < nrc) ++lg;
        MfmaApplyDev d{};
        d.nrc = nrc;
        d.lg_nrc = lg;
        d.ncur = ncur;
        d.ldx = nrhs;
        d.ldy = nrhs;
        d.c0 = c0;
        std::vector<int64_t> zoff(std::max<int64_t>(nfar, 1), 0);
        int64_t zacc = 0;
        for (int64_t b = 0; b < nfar; ++b) {
            zoff[b] = zacc;
            zacc += (int64_t)sum_rho[b] * nrc;
        }
        h->d_mzoff.upload(ctx, zoff);
        d.z_off = h->d_mzoff.as<int64_t>();
        d.sum_rho = h->d_msumrho.as<int32_t>();
        for (size_t g0 = 0; g0 < groups.size();) {
            std::vector<MfmaTGroup> tg;
            std::vector<int64_t> tt0;
            std::vector<MfmaTRow> trows;
            std::vector<MfmaZItem> zi;
            int64_t tacc = 0, ntiles = 0;
            size_t g1 = g0;
            for (; g1 < groups.size(); ++g1) {
                const auto &grp = groups[g1];
                const int n = (int)p->part.far[grp[0]][3];
                int64_t rows = 0;
                for (int64_t e : grp) rows += h->meta[e].rank;
                const int64_t tg_bytes = rows * n * nrc * (int64_t)sizeof(float2);
                if (g1 > g0 && (size_t)(tacc * sizeof(float2) + tg_bytes) > t_budget) break;
                if (rows == 0) continue;
                MfmaTGroup G{};
                G.c0 = (int32_t)p->part.far[grp[0]][2];
                G.n = n;
                G.rows = (int32_t)rows;
                G.m_tiles = (int32_t)((rows + 31) / 32);
                G.row0 = (int64_t)trows.size();
                tt0.push_back(ntiles);
                tg.push_back(G);
                ntiles += (int64_t)G.m_tiles * (((int64_t)n * nrc + 255) / 256);
                for (int64_t e : grp) {
                    const FarMeta &mt = h->meta[e];
                    if (mt.rank == 0) continue;
                    const int64_t t_b = tacc;
                    int64_t qoff = 0;
                    for (int l = 0; l < mt.rank; ++l) {
                        trows.push_back(MfmaTRow{h->fib_off[e] + (int64_t)l * p->L, t_b + (int64_t)l * n * nrc});
                        const CrossMeta &cm = h->cmeta[e * h->rcap + l];
                        for (int q0 = 0; q0 < cm.rho; q0 += 32) {
                            MfmaZItem z{};
                            z.b = (int32_t)e;
                            z.l = l;
                            z.q0 = q0;
                            z.t_off = t_b;
                            z.z_off = zoff[e] + qoff * nrc;
                            zi.push_back(z);
                        }
                        qoff += cm.rho;
                    }
                    tacc += (int64_t)mt.rank * n * nrc;
                }
            }
            if (!tg.empty()) {
                ensure(ctx, h->d_mt, (size_t)std::max<int64_t>(tacc, 1) * sizeof(float2));
                h->d_mtitems.upload(ctx, tg);
                h->d_mttile0.upload(ctx, tt0);
                h->d_mtrows.upload(ctx, trows);
                h->d_mzitems.upload(ctx, zi);
                d.t_groups = h->d_mtitems.as<MfmaTGroup>();
                d.t_tile0 = h->d_mttile0.as<int64_t>();
                d.nt_groups = (int32_t)tg.size();
                d.t_rows = h->d_mtrows.as<MfmaTRow>();
                d.z_items = h->d_mzitems.as<MfmaZItem>();
                GACA_HIP_CHECK(hipEventRecord(ep[0], st));
                launch_apply_far_t(a, d, ntiles, X, h->d_mt.as<float2>(), st);
                GACA_HIP_CHECK(hipEventRecord(ep[1], st));
                launch_apply_far_z(a, d, (int)zi.size(), h->d_mt.as<float2>(), h->d_mz.as<float2>(), st);
                GACA_HIP_CHECK(hipEventRecord(ep[2], st));
                GACA_HIP_CHECK(hipGetLastError());
                // the next batch reuses T and the item lists
                GACA_HIP_CHECK(hipStreamSynchronize(st));
                ms_part[0] += part_ms(0, 1);
                ms_part[1] += part_ms(1, 2);
            }
            g0 = g1;
        }
        GACA_HIP_CHECK(hipEventRecord(ep[2], st));
        launch_apply_leaf_mfma(a, d, row_tiles, X, h->d_mz.as<float2>(), Y, st);
        GACA_HIP_CHECK(hipEventRecord(ep[3], st));
        GACA_HIP_CHECK(hipGetLastError());
        // the next chunk rewrites Z and the offsets
        GACA_HIP_CHECK(hipStreamSynchronize(st));
        ms_part[2] += part_ms(2, 3);
    }
    GACA_HIP_CHECK(hipEventRecord(ev1, st));
    GACA_HIP_CHECK(hipEventSynchronize(ev1));
    float ms = 0.0f;
    GACA_HIP_CHECK(hipEventElapsedTime(&ms, ev0, ev1));
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    for (auto &e : ep) (void)hipEventDestroy(e);
    h->st.ms_apply = ms;
    for (int k = 0; k < 3; ++k) h->st.ms_apply_part[k] = ms_part[k];
}

// Device view of an operator for the apply kernels (workspace offsets and the T group size
// are set by the caller).
static ApplyDev apply_view(gaca_hmatrix *h, int32_t nrhs) {
    gaca_problem *p = h->p;
    ApplyDev a{};
    a.L = p->L;
    a.nrhs = nrhs;
    a.M = p->M;
    a.perm = p->d_perm.as<int64_t>();
    a.nfar = (int32_t)h->nfar;
    a.nnear = (int32_t)p->nblocks.size();
    a.rcap = h->rcap;
    a.far4 = h->d_far4.as<int32_t>();
    a.meta = h->d_meta.as<FarMeta>();
    a.cmeta = h->d_cmeta.as<CrossMeta>();
    a.cross_off = h->d_cross_off.as<int64_t>();
    a.arena = h->d_arena.ptr;
    a.fac_fp32 = h->prec == GACA_MIXED ? 1 : 0;
    a.fib_off = h->d_fib_off.as<int64_t>();
    a.fib_arena = h->d_fib.as<double2>();
    if (h->near_aca) {
        // compressed near blocks: the operator's own block table; dense ones in the compact arena
        a.nblocks = h->d_nblk_own.as<NearBlockDev>();
        a.near64 = h->prec == GACA_MIXED ? nullptr : h->n_dense.as<double2>();
        a.near32 = h->prec == GACA_MIXED ? h->n_dense.as<float2>() : nullptr;
        a.near_faces = h->n_faces.ptr;
        a.near_fib = h->n_fib.as<double2>();
        a.tn_off = h->d_tnoff.as<int64_t>();
    } else {
        a.nblocks = p->d_nblocks.as<NearBlockDev>();
        a.near64 = h->prec == GACA_MIXED ? nullptr : h->d_near.as<double2>();
        a.near32 = h->prec == GACA_MIXED ? h->d_near.as<float2>() : nullptr;
    }
    a.nleaf = (int32_t)p->leaf_r0.size();
    a.max_leaf_m = 1;
    for (int32_t lm : p->leaf_m) a.max_leaf_m = std::max(a.max_leaf_m, lm);
    a.leaf_r0 = p->d_leaf_r0.as<int32_t>();
    a.leaf_m = p->d_leaf_m.as<int32_t>();
    a.leaf_far_ptr = p->d_lfp.as<int32_t>();
    a.leaf_far_idx = p->d_lfi.as<int32_t>();
    a.leaf_near_ptr = p->d_lnp.as<int32_t>();
    a.leaf_near_idx = p->d_lni.as<int32_t>();
    return a;
}

gaca_status gaca_apply(gaca_hmatrix *h, gaca_apply_mode mode, int32_t nrhs, const void *X,
                       void *Y, gaca_dtype dtype, void *hip_stream) {
    return guarded([&] {
        REQUIRE(h && X && Y, "null argument");
        REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        REQUIRE(mode == GACA_APPLY_SUM || mode == GACA_APPLY_PER_FREQ, "bad mode");
        REQUIRE(dtype == GACA_C128 || dtype == GACA_C64, "bad dtype");
        REQUIRE(!h->p->synthetic, "apply needs a mesh problem");
        gaca_problem *p = h->p;
        gaca_context *ctx = p->ctx;
        hipStream_t st = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : ctx->stream;
        prepare_leaves(h);
        const int L = p->L;
        const int64_t M = p->M;
        const size_t xs = dtype == GACA_C64 ? sizeof(float2) : sizeof(double2);
        // matrix cores from kMfmaMinRhs right-hand sides on (below, their 16-column tiles are
        // mostly padding and the VALU apply is faster)
        const bool mfma = mode == GACA_APPLY_SUM && dtype == GACA_C64 && nrhs >= kMfmaMinRhs &&
                          mfma_supported(h);
        if (!mfma && (h->ws_nrhs != nrhs || h->ws_mode != (int)mode || h->ws_dtype != (int)dtype))
            alloc_apply_workspace(h, mode, nrhs, dtype);
        ApplyDev a = apply_view(h, nrhs);
        a.apply_cb = h->ws_cb;
        a.z_off = h->d_zoff.as<int64_t>();
        if (mfma) {
            apply_mfma(h, a, nrhs, reinterpret_cast<const float2 *>(X), reinterpret_cast<float2 *>(Y), st);
            return;
        }
        // SUM mode: the far blocks on one of the problem's far-field streams (idle between
        // builds) beside the near part of the leaf sums
        ApplySide side{};
        const bool use_side = mode == GACA_APPLY_SUM && p->far_streams_ready && h->nfar > 0;
        if (use_side) {
            for (hipEvent_t &e : h->apply_ev)
                if (!e) GACA_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            side.stream = p->far_streams[1];
            side.fork = h->apply_ev[0];
            side.join = h->apply_ev[1];
        }
        launch_apply(a, (int)mode, dtype == GACA_C64 ? 1 : 0, X, Y, h->d_xp.ptr, h->d_yp.ptr,
                     h->d_z.ptr, h->d_t.ptr, h->d_toff.as<int64_t>(), h->d_yb.ptr,
                     h->d_yoff.as<int64_t>(), st, h->d_tn.ptr, use_side ? &side : nullptr);
        GACA_HIP_CHECK(hipGetLastError());
    });
}

gaca_status gaca_apply_noalloc(gaca_hmatrix *h, gaca_apply_mode mode, int32_t nrhs, const void *X,
                               void *Y, gaca_dtype dtype, void *hip_stream) {
    return guarded([&] {
        REQUIRE(h && X && Y, "null argument");
        REQUIRE(nrhs >= 1, "nrhs must be >= 1");
        REQUIRE(mode == GACA_APPLY_SUM || mode == GACA_APPLY_PER_FREQ, "bad mode");
        REQUIRE(dtype == GACA_C128 || dtype == GACA_C64, "bad dtype");
        REQUIRE(!h->p->synthetic, "apply needs a mesh problem");
        gaca_problem *p = h->p;
        gaca_context *ctx = p->ctx;
        if (!p->leaf_ready) throw Error{GACA_ERR_STATE, "leaf tables missing (built with the operator)"};
        if (h->near_aca)
            throw Error{GACA_ERR_UNSUPPORTED, "the allocation-free apply takes dense near fields (near_aca = 0)"};
        void *base = scratch_address(ctx->device);
        if (!base) throw Error{GACA_ERR_STATE, "scratch array not set up on this device"};
        hipStream_t st = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : ctx->stream;
        const int L = p->L;
        const int64_t M = p->M;
        const size_t xs = dtype == GACA_C64 ? sizeof(float2) : sizeof(double2);
        const int cb = kApplyCB;
        // workspace sizes (elements), as the allocated workspace of gaca_apply
        int64_t zacc = 0, tacc = 0, yacc = 0;
        for (int64_t b = 0; b < h->nfar; ++b) {
            const int64_t sr = h->meta[b].sum_rho;
            yacc += p->part.far[b][1] * (int64_t)nrhs;
            zacc += mode == GACA_APPLY_SUM ? sr * nrhs : sr * (int64_t)L * nrhs;
            if (mode == GACA_APPLY_SUM)
                tacc += std::min<int64_t>(h->meta[b].rank, cb) * p->part.far[b][3] * (int64_t)nrhs;
        }
        const int nl = mode == GACA_APPLY_SUM ? 1 : L;
        auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
        const size_t o_off = 0;
        const size_t o_xp = al(o_off + 3 * (size_t)std::max<int64_t>(h->nfar, 1) * sizeof(int64_t));
        const size_t o_yp = al(o_xp + (size_t)L * M * nrhs * xs);
        const size_t o_z = al(o_yp + (size_t)nl * M * nrhs * xs);
        const size_t o_t = al(o_z + (size_t)std::max<int64_t>(zacc, 1) * xs);
        const size_t o_yb = al(o_t + (size_t)std::max<int64_t>(tacc, 1) * xs);
        const size_t need = al(o_yb + (size_t)std::max<int64_t>(yacc, 1) * xs);
        if (need > kScratchBytes)
            throw Error{GACA_ERR_INVALID_ARG,
                        "apply workspace of " + std::to_string(need) + " bytes exceeds the " +
                            std::to_string(kScratchBytes) + "-byte scratch array of the allocation-free apply"};
        unsigned char *sb = static_cast<unsigned char *>(base);
        int64_t *zoff = reinterpret_cast<int64_t *>(sb + o_off);
        int64_t *toff = zoff + std::max<int64_t>(h->nfar, 1);
        int64_t *yoff = toff + std::max<int64_t>(h->nfar, 1);
        ApplyDev a = apply_view(h, nrhs);
        a.apply_cb = cb;
        a.z_off = zoff;
        launch_apply_offsets(a, (int)mode, cb, zoff, toff, yoff, st);
        launch_apply(a, (int)mode, dtype == GACA_C64 ? 1 : 0, X, Y, sb + o_xp, sb + o_yp, sb + o_z,
                     sb + o_t, toff, sb + o_yb, yoff, st);
        GACA_HIP_CHECK(hipGetLastError());
    });
}

// ---------------------------------------------------------------------------------------
// gCQ (Sec. 3 temporal discretisation, App. A)
gaca_status gaca_gcq_contour(int32_t stages, const double *rk_A, double dt_min, double dt_max,
                             int32_t n_q, double *s_re, double *s_im, double *w_re,
                             double *w_im) {
    return guarded([&] {
        REQUIRE(rk_A && s_re && s_im && w_re && w_im, "null argument");
        REQUIRE(stages >= 1 && stages <= kGcqMaxStages, "stages must be in [1, 4]");
        REQUIRE(n_q >= 1 && n_q <= 1 << 20, "n_q out of range");
        REQUIRE(std::isfinite(dt_min) && std::isfinite(dt_max) && dt_min > 0.0 && dt_max >= dt_min,
                "need 0 < dt_min <= dt_max");
        for (int i = 0; i < stages * stages; ++i) REQUIRE(std::isfinite(rk_A[i]), "non-finite Butcher matrix");
        gcq_contour(stages, rk_A, dt_min, dt_max, n_q, s_re, s_im, w_re, w_im);
    });
}

gaca_status gaca_gcq_history(gaca_hmatrix *h, int32_t stages, const double *rk_A,
                             const double *rk_b, double dt_prev, double dt_cur,
                             const double *w_re, const double *w_im, const void *theta_prev,
                             void *x, void *W, void *Y, void *hip_stream) {
    const gaca_status rc = guarded([&] {
        REQUIRE(h && rk_A && rk_b && w_re && w_im && theta_prev && x && W && Y, "null argument");
        REQUIRE(!h->p->synthetic, "the history step needs a mesh problem");
        REQUIRE(stages >= 1 && stages <= kGcqMaxStages, "stages must be in [1, 4]");
        REQUIRE(std::isfinite(dt_prev) && std::isfinite(dt_cur) && dt_prev > 0.0 && dt_cur > 0.0,
                "step sizes must be positive");
        gaca_problem *p = h->p;
        gaca_context *ctx = p->ctx;
        hipStream_t st = hip_stream ? reinterpret_cast<hipStream_t>(hip_stream) : ctx->stream;
        const int m = stages;
        GcqDev q{};
        q.L = p->L;
        q.m = m;
        q.M = p->M;
        q.dt_prev = dt_prev;
        q.dt_cur = dt_cur;
        for (int i = 0; i < m * m; ++i) q.A[i] = rk_A[i];
        // g = b^T A^{-1}: solve A^T g = b (Gaussian elimination, partial pivoting)
        double T[kGcqMaxStages][kGcqMaxStages + 1];
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < m; ++j) T[i][j] = rk_A[j * m + i];
            T[i][m] = rk_b[i];
        }
        for (int c = 0; c < m; ++c) {
            int pv = c;
            for (int r = c + 1; r < m; ++r)
                if (std::fabs(T[r][c]) > std::fabs(T[pv][c])) pv = r;
            REQUIRE(std::fabs(T[pv][c]) > 0.0, "the Butcher matrix is singular");
            for (int j = 0; j <= m; ++j) std::swap(T[c][j], T[pv][j]);
            for (int r = c + 1; r < m; ++r) {
                const double f = T[r][c] / T[c][c];
                for (int j = c; j <= m; ++j) T[r][j] -= f * T[c][j];
            }
        }
        for (int c = m - 1; c >= 0; --c) {
            double v = T[c][m];
            for (int j = c + 1; j < m; ++j) v -= T[c][j] * q.g[j];
            q.g[c] = v / T[c][c];
        }
        // quadrature weights on the device (kept by the operator, rewritten per call)
        std::vector<double> wv(2 * (size_t)p->L);
        for (int l = 0; l < p->L; ++l) {
            REQUIRE(std::isfinite(w_re[l]) && std::isfinite(w_im[l]), "non-finite weight");
            wv[l] = w_re[l];
            wv[p->L + l] = w_im[l];
        }
        if (!h->d_gcqw.ptr) h->d_gcqw.alloc(ctx, wv.size() * sizeof(double));
        GACA_HIP_CHECK(hipMemcpyAsync(h->d_gcqw.ptr, wv.data(), wv.size() * sizeof(double),
                                      hipMemcpyHostToDevice, st));
        q.w_re = h->d_gcqw.as<double>();
        q.w_im = q.w_re + p->L;
        launch_gcq_history(q, p->f.re, p->f.im, static_cast<const double2 *>(theta_prev),
                           static_cast<double2 *>(x), static_cast<double2 *>(W), st);
        GACA_HIP_CHECK(hipGetLastError());
        // the host copy of the weights must outlive the asynchronous copy
        GACA_HIP_CHECK(hipStreamSynchronize(st));
    });
    if (rc != GACA_OK) return rc;
    // history term sum_l V(s_l) W_l: the reordered product with the stages as right-hand sides
    return gaca_apply(h, GACA_APPLY_SUM, stages, W, Y, GACA_C128, hip_stream);
}

// ---------------------------------------------------------------------------------------
gaca_status gaca_eval_entries(gaca_problem *p, gaca_kernel kernel, int64_t n, const int32_t *i,
                              const int32_t *j, const int32_t *k, const int32_t *far,
                              double *out) {
    return guarded([&] {
        REQUIRE(p, "null problem");
        REQUIRE(kernel == GACA_SLP || kernel == GACA_DLP || kernel == GACA_HYP || kernel == GACA_ADLP,
                "bad kernel");
        REQUIRE(n >= 0, "n must be >= 0");
        if (n == 0) return;
        REQUIRE(i && j && k && far && out, "null argument");
        REQUIRE(!p->synthetic, "entries need a mesh problem");
        std::vector<int32_t> rows(n), cols(n), ks(n), tiers(n);
        if (p->scheme == GACA_COLLOCATION_P1 && kernel != GACA_DLP)
            throw Error{GACA_ERR_UNSUPPORTED, "the P1 scheme has the double layer only"};
        if ((p->scheme == GACA_GALERKIN_P1) != (kernel == GACA_HYP || kernel == GACA_ADLP))
            throw Error{GACA_ERR_UNSUPPORTED,
                        "the hypersingular operator and the adjoint double layer belong to the Galerkin P1 scheme"};
        for (int64_t t = 0; t < n; ++t) {
            REQUIRE(i[t] >= 0 && i[t] < p->M && j[t] >= 0 && j[t] < p->M, "element id out of range");
            REQUIRE(k[t] >= 0 && k[t] < p->L, "frequency index out of range");
            rows[t] = (int32_t)p->inv_perm[i[t]];
            cols[t] = (int32_t)p->inv_perm[j[t]];
            ks[t] = k[t];
            if (p->p1())
                tiers[t] = far[t] ? 1 : 0;   // the far flag (tiers are chosen per triangle)
            else if (p->scheme == GACA_GALERKIN_P0)
                tiers[t] = i[t] == j[t] ? 5 : (far[t] ? 0 : galerkin_tier(p->mesh, i[t], j[t]));
            else
                tiers[t] = far[t] ? (i[t] == j[t] ? TIER_SELF : TIER_FAR6)
                                  : collocation_tier(p->mesh, i[t], j[t]);
        }
        if (p->scheme == GACA_GALERKIN_P0 && kernel != GACA_SLP)
            throw Error{GACA_ERR_UNSUPPORTED, "Galerkin is available for the single layer only"};
        gaca_context *ctx = p->ctx;
        DevBuf dr, dc, dk, dt, dout;
        dr.upload(ctx, rows);
        dc.upload(ctx, cols);
        dk.upload(ctx, ks);
        dt.upload(ctx, tiers);
        dout.alloc(ctx, n * sizeof(double2));
        if (p->scheme == GACA_COLLOCATION_P1)
            launch_eval_p1(p->g, p->q, p->f, n, dr.as<int32_t>(), dc.as<int32_t>(), dk.as<int32_t>(),
                           dt.as<int32_t>(), dout.as<double2>(), ctx->stream);
        else if (p->scheme == GACA_GALERKIN_P1)
            launch_eval_gp1(kernel == GACA_HYP ? 0 : 1, p->g, p->q, p->f, n, dr.as<int32_t>(), dc.as<int32_t>(),
                            dk.as<int32_t>(), dt.as<int32_t>(), dout.as<double2>(), ctx->stream);
        else
            launch_eval(p->kid(kernel), p->g, p->q, p->f, n, dr.as<int32_t>(), dc.as<int32_t>(),
                        dk.as<int32_t>(), dt.as<int32_t>(), dout.as<double2>(), ctx->stream);
        GACA_HIP_CHECK(hipGetLastError());
        GACA_HIP_CHECK(hipStreamSynchronize(ctx->stream));
        GACA_HIP_CHECK(hipMemcpy(out, dout.ptr, n * sizeof(double2), hipMemcpyDeviceToHost));
    });
}

gaca_status gaca_eval_far_entries_mixed(gaca_problem *p, gaca_kernel kernel, int64_t far_block,
                                        int64_t n, const int32_t *il, const int32_t *jl,
                                        const int32_t *k, double *out) {
    return guarded([&] {
        REQUIRE(p, "null problem");
        REQUIRE(kernel == GACA_SLP || kernel == GACA_DLP, "bad kernel");
        REQUIRE(!p->synthetic, "entries need a mesh problem");
        REQUIRE(far_block >= 0 && far_block < (int64_t)p->part.far.size(), "far block index out of range");
        REQUIRE(n >= 0, "n must be >= 0");
        if (n == 0) return;
        REQUIRE(il && jl && k && out, "null argument");
        if (p->scheme == GACA_GALERKIN_P0 && kernel != GACA_SLP)
            throw Error{GACA_ERR_UNSUPPORTED, "Galerkin is available for the single layer only"};
        if (p->p1())
            throw Error{GACA_ERR_UNSUPPORTED, "the P1 operators have no mixed-precision path"};
        const auto &fb = p->part.far[far_block];
        FarBlockDev d{};
        d.r0 = (int32_t)fb[0];
        d.m = (int32_t)fb[1];
        d.c0 = (int32_t)fb[2];
        d.n = (int32_t)fb[3];
        d.kern = kernel;
        set_far_scaling(p, far_block, d);
        std::vector<int32_t> a(n), b(n), c(n);
        for (int64_t t = 0; t < n; ++t) {
            REQUIRE(il[t] >= 0 && il[t] < d.m && jl[t] >= 0 && jl[t] < d.n, "local index out of range");
            REQUIRE(k[t] >= 0 && k[t] < p->L, "frequency index out of range");
            a[t] = il[t];
            b[t] = jl[t];
            c[t] = k[t];
        }
        gaca_context *ctx = p->ctx;
        DevBuf da, db, dc, dout;
        da.upload(ctx, a);
        db.upload(ctx, b);
        dc.upload(ctx, c);
        dout.alloc(ctx, n * sizeof(double2));
        launch_eval_far_mixed(p->kid(kernel), p->g, p->f, d, n, da.as<int32_t>(), db.as<int32_t>(),
                              dc.as<int32_t>(), dout.as<double2>(), ctx->stream);
        GACA_HIP_CHECK(hipGetLastError());
        GACA_HIP_CHECK(hipStreamSynchronize(ctx->stream));
        GACA_HIP_CHECK(hipMemcpy(out, dout.ptr, n * sizeof(double2), hipMemcpyDeviceToHost));
    });
}

gaca_status gaca_compress_tensor(gaca_context *ctx, const void *dev_tensor, int64_t m,
                                 int64_t n, int32_t L, const gaca_options *opt,
                                 gaca_hmatrix **out) {
    bool capped = false;
    gaca_status rc = guarded([&] {
        REQUIRE(ctx && dev_tensor && out, "null argument");
        REQUIRE(m >= 1 && n >= 1 && m <= 8192 && n <= 8192, "tensor sides must be in [1, 8192]");
        REQUIRE(L >= 1 && L <= 1024, "L must be in [1, 1024]");
        auto p = std::make_unique<gaca_problem>();
        p->attach(ctx);
        if (opt) p->opt = *opt;
        else options_default(&p->opt);
        p->opt.autotune_cache = nullptr;
        if (p->opt.precision != GACA_FP64)
            throw Error{GACA_ERR_UNSUPPORTED, "compress_tensor runs in FP64"};
        p->synthetic = true;
        p->M = std::max(m, n);
        p->L = L;
        p->part.far.push_back({0, m, 0, n});
        p->f.L = L;
        p->f.L_eval = L;
        p->f.mirror = 0;
        std::vector<double> dummy(2 * L, 0.0);
        p->d_freq.upload(ctx, dummy);
        p->f.re = p->d_freq.as<double>();
        p->f.im = p->d_freq.as<double>() + L;
        auto h = std::make_unique<gaca_hmatrix>();
        h->p = p.get();
        h->kernel = 0;
        h->prec = GACA_FP64;
        h->rcap = std::max(1, std::min({L, p->opt.max_rank3d > 0 ? p->opt.max_rank3d : L, 256}));
        GACA_HIP_CHECK(hipSetDevice(ctx->device));
        run_far({h.get()}, reinterpret_cast<const double2 *>(dev_tensor), [] {});
        fill_stats(h.get());
        capped = h->st.n_capped > 0;
        h->owned_problem = std::move(p);
        *out = h.release();
    });
    if (rc == GACA_OK && capped) {
        set_error("rank cap hit");
        return GACA_ERR_NOT_CONVERGED;
    }
    return rc;
}

}  // extern "C"
