// C ABI of libgaca (include/gaca.h): context, problem (mesh, frequencies, tree,
// partition, device geometry), build (near field + far-field 3D-ACA), export, apply.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <functional>
#include <numeric>

#include "host.h"
#include "kernels.h"

using namespace gaca;

// ---------------------------------------------------------------------------------------
// device buffers with accounting against max_device_bytes
struct gaca_context {
    int device = 0;
    hipStream_t stream = nullptr;
    uint64_t limit = 0;       // 0: none
    uint64_t in_use = 0;
};

namespace {

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
        hipError_t e = hipMalloc(&ptr, nbytes);
        if (e != hipSuccess) {
            ptr = nullptr;
            (void)hipGetLastError();
            throw Error{GACA_ERR_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
        }
        bytes = nbytes;
        c->in_use += nbytes;
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

struct gaca_problem {
    gaca_context *ctx = nullptr;
    gaca_options opt{};
    gaca_scheme scheme = GACA_COLLOCATION_P0;
    bool synthetic = false;       // dense-tensor problem of gaca_compress_tensor
    HostMesh mesh;
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
    int kid(gaca_kernel k) const { return scheme == GACA_GALERKIN_P0 ? 2 : (int)k; }
    // leaves for the apply
    std::vector<int32_t> leaf_r0, leaf_m;
    // far-field launch classes run concurrently on these streams (default priority)
    hipStream_t far_streams[3] = {nullptr, nullptr, nullptr};
    bool far_streams_ready = false;
    ~gaca_problem() {
        if (far_streams_ready)
            for (auto &s : far_streams) (void)hipStreamDestroy(s);
    }
};

struct gaca_hmatrix {
    gaca_problem *p = nullptr;
    std::unique_ptr<gaca_problem> owned_problem;   // synthetic problems
    int kernel = 0;
    gaca_precision prec = GACA_FP64;
    int32_t rcap = 0;
    int64_t nfar = 0;
    double eps_aca_used = 0.0;
    DevBuf d_near, d_arena, d_fib, d_meta, d_cmeta, d_cross_off, d_fib_off, d_far4;
    std::vector<FarMeta> meta;
    std::vector<CrossMeta> cmeta;
    std::vector<int64_t> cross_off, fib_off;
    gaca_stats st{};
    std::vector<int64_t> freq_hist;
    // apply workspace
    int32_t ws_nrhs = -1, ws_mode = -1, ws_dtype = -1;
    DevBuf d_xp, d_yp, d_z, d_t, d_toff, d_zoff, d_yb, d_yoff;
    DevBuf d_leaf_r0, d_leaf_m, d_lfp, d_lfi, d_lnp, d_lni;
    bool leaf_ready = false;
};

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
        auto *c = new gaca_context;
        c->device = device;
        c->stream = reinterpret_cast<hipStream_t>(hip_stream);
        *out = c;
    });
}

gaca_status gaca_context_destroy(gaca_context *ctx) {
    delete ctx;
    return GACA_OK;
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
        *n_far = (int64_t)part.far.size();
        *n_near = (int64_t)part.near.size();
        if ((int64_t)part.far.size() > capacity || (int64_t)part.near.size() > capacity)
            throw Error{GACA_ERR_INVALID_ARG, "block list capacity too small"};
        for (size_t b = 0; b < part.far.size(); ++b)
            for (int k = 0; k < 4; ++k) far4[4 * b + k] = part.far[b][k];
        for (size_t b = 0; b < part.near.size(); ++b)
            for (int k = 0; k < 4; ++k) near4[4 * b + k] = part.near[b][k];
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

static void upload_problem(gaca_problem *p) {
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
    // quadrature tables
    Rule1D r4 = gauss_legendre01(4), r8 = gauss_legendre01(8),
           rd = gauss_legendre01(p->opt.n_duffy), rg = gauss_legendre01(p->opt.n_galerkin);
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
           oth = push_rule(rth);
    size_t o6 = qt.size();
    for (int q = 0; q < 6; ++q) {
        qt.push_back(bary[q][0]);
        qt.push_back(bary[q][1]);
        qt.push_back(bary[q][2]);
        qt.push_back(w6[q]);
    }
    p->d_quad.upload(ctx, qt);
    const double *Q = p->d_quad.as<double>();
    p->q.n4 = 4;
    p->q.n8 = 8;
    p->q.nd = p->opt.n_duffy;
    p->q.ng = p->opt.n_galerkin;
    p->q.g4 = Q + o4;
    p->q.g8 = Q + o8;
    p->q.gd = Q + od;
    p->q.gg = Q + og;
    p->q.r6 = Q + o6;
    p->q.nth = kGalerkinNTheta;
    p->q.gth = Q + oth;
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
    // leaves in tree order
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
        REQUIRE(scheme == GACA_COLLOCATION_P0 || scheme == GACA_GALERKIN_P0, "bad scheme");
        auto p = std::make_unique<gaca_problem>();
        p->ctx = ctx;
        if (opt) p->opt = *opt;
        else options_default(&p->opt);
        REQUIRE(p->opt.eta > 0.0, "eta must be > 0");
        REQUIRE(p->opt.eps3d >= 0.0 && p->opt.eps_aca >= 0.0, "tolerances must be >= 0");
        REQUIRE(p->opt.n_duffy >= 1 && p->opt.n_duffy <= 64, "n_duffy out of range");
        REQUIRE(p->opt.n_galerkin >= 1 && p->opt.n_galerkin <= 32, "n_galerkin out of range");
        REQUIRE(p->opt.tie >= 0.0 && p->opt.tie < 1.0, "tie out of range");
        ctx->limit = p->opt.max_device_bytes;
        p->scheme = scheme;
        p->mesh.init(xyz, nv, tri, M);
        p->M = M;
        p->L = L;
        p->s_re.assign(s_re, s_re + L);
        p->s_im.assign(s_im, s_im + L);
        for (int l = 0; l < L; ++l)
            REQUIRE(std::isfinite(s_re[l]) && std::isfinite(s_im[l]), "non-finite frequency");
        bool mir = true;
        for (int l = 0; l < L; ++l)
            if (!(s_re[L - 1 - l] == s_re[l] && s_im[L - 1 - l] == -s_im[l])) mir = false;
        p->mirror = mir;
        p->tree.build(p->mesh, p->opt.leaf_size);
        p->part.build(p->tree, p->opt.eta);
        p->inv_perm.assign(M, 0);
        for (int64_t t = 0; t < M; ++t) p->inv_perm[p->tree.perm[t]] = t;
        GACA_HIP_CHECK(hipSetDevice(ctx->device));
        upload_problem(p.get());
        upload_freq(p.get());
        *out = p.release();
    });
}

gaca_status gaca_problem_destroy(gaca_problem *p) {
    delete p;
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
// Launch class of a far block: small blocks keep the residual face in LDS.
static int far_kind(int m, int n, int rcap) {
    const int64_t mn = (int64_t)m * n;
    if (rcap <= 64 && mn <= 1024 && m <= 64 && n <= 64) return 0;
    if (rcap <= 64 && mn <= 2304 && m <= 96 && n <= 96) return 1;
    return 2;
}

// Replace buf by a copy holding its first `used` bytes when that frees a useful amount.
static void compact(gaca_context *ctx, DevBuf &buf, size_t used, hipStream_t st) {
    if (used == 0 || buf.bytes < (64u << 20) || used > buf.bytes / 4 * 3) return;
    DevBuf tight;
    tight.alloc(ctx, used);
    GACA_HIP_CHECK(hipMemcpyAsync(tight.ptr, buf.ptr, used, hipMemcpyDeviceToDevice, st));
    GACA_HIP_CHECK(hipStreamSynchronize(st));
    std::swap(buf.ptr, tight.ptr);
    std::swap(buf.bytes, tight.bytes);
}

static void run_far(gaca_hmatrix *h, const double2 *dense, const std::function<void()> &main_work) {
    gaca_problem *p = h->p;
    gaca_context *ctx = p->ctx;
    const auto &far = p->part.far;
    const int64_t nfar = (int64_t)far.size();
    h->nfar = nfar;
    const int L = p->L;
    const int rcap = h->rcap;
    const hipStream_t st = ctx->stream;
    h->meta.assign(nfar, FarMeta{});
    h->cmeta.assign(nfar * rcap, CrossMeta{});
    h->cross_off.assign(nfar * rcap, -1);
    h->fib_off.assign(nfar, -1);
    std::vector<int32_t> far4(4 * std::max<int64_t>(nfar, 1));
    for (int64_t b = 0; b < nfar; ++b)
        for (int k = 0; k < 4; ++k) far4[4 * b + k] = (int32_t)far[b][k];
    h->d_far4.upload(ctx, far4);
    if (nfar == 0) {
        main_work();
        return;
    }
    h->d_meta.alloc(ctx, nfar * sizeof(FarMeta));
    h->d_cmeta.alloc(ctx, nfar * rcap * sizeof(CrossMeta));
    h->d_cross_off.alloc(ctx, nfar * rcap * sizeof(int64_t));
    h->d_fib_off.alloc(ctx, nfar * sizeof(int64_t));
    // per-block scratch (complex elements) and launch classes
    struct Item {
        int64_t b, bytes;
        int kind;
        FarBlockDev d;
    };
    std::vector<Item> items;
    double factor_guess = 0.0;
    for (int64_t b = 0; b < nfar; ++b) {
        const int m = (int)far[b][1], n = (int)far[b][3];
        if (m > 8192) throw Error{GACA_ERR_UNSUPPORTED, "far block with more than 8192 rows"};
        int rho_max = std::min(m, n);
        if (p->opt.max_face_rank > 0) rho_max = std::min(rho_max, p->opt.max_face_rank);
        FarBlockDev d{};
        d.r0 = (int32_t)far[b][0];
        d.m = m;
        d.c0 = (int32_t)far[b][2];
        d.n = n;
        d.rho_max = rho_max;
        d.out_idx = (int32_t)b;
        // scratch layout in bytes: faces and current-face factors in the face type, fibres
        // and Gram values in double2 (16-byte aligned)
        const int64_t es = h->prec == GACA_MIXED ? 8 : 16;
        auto al16 = [](int64_t v) { return (v + 15) & ~(int64_t)15; };
        int64_t faces = al16((int64_t)rcap * m * n * es), uw = al16((int64_t)rho_max * (m + n) * es),
                fibs = (int64_t)rcap * L * 16, gram = (int64_t)rcap * rcap * 16;
        d.face_off = 0;
        d.uw_off = faces;
        d.fib_off = faces + uw;
        d.gram_off = faces + uw + fibs;
        if (!p->synthetic && p->part.far_nodes.size() == far.size()) {
            // mixed scaling geometry from the cluster boxes
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
        items.push_back(Item{b, faces + uw + fibs + gram, far_kind(m, n, rcap), d});
        // first guess of the factor storage: 16 crosses of face rank 16, never more than
        // the dense block (the build retries with a larger arena when the guess is short)
        factor_guess += std::min((double)m * n * L,
                                 (double)std::min(rcap, 16) * std::min(rho_max, 16) * (m + n));
    }
    // large blocks first, biggest first inside each class
    std::stable_sort(items.begin(), items.end(), [](const Item &a, const Item &b) {
        if (a.kind != b.kind) return a.kind > b.kind;
        return a.bytes > b.bytes;
    });
    const size_t fac_bytes = h->prec == GACA_MIXED ? sizeof(float2) : sizeof(double2);
    uint64_t arena_cap = (uint64_t)std::max(1.0e6, factor_guess);
    uint64_t fib_cap = (uint64_t)std::max<int64_t>(1 << 16, nfar * (int64_t)std::min(rcap, 16) * L);
    {
        // keep the first guess within a third of the free device memory
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && free_b > 0)
            arena_cap = std::min<uint64_t>(arena_cap, std::max<uint64_t>(1 << 20, free_b / 3 / fac_bytes));
    }
    const uint64_t budget_elems = std::max<uint64_t>(p->opt.batch_bytes / 3, 16ull << 20);  // bytes
    AcaParams P{};
    P.eps = p->opt.eps3d;
    P.eps_aca = p->opt.eps_aca;
    P.tie = p->opt.tie;
    P.delta = p->opt.delta_zero;
    if (h->prec == GACA_MIXED) {
        // FP32 faces: the face tolerance, tie window and zero threshold cannot go below
        // what FP32 resolves
        P.eps_aca = std::max(P.eps_aca, 2e-6);
        P.tie = std::max(P.tie, 1e-4);
        P.delta = std::max(P.delta, 1e-6);
    }
    h->eps_aca_used = P.eps_aca;
    P.rcap = rcap;
    P.kernel = h->kernel;
    DevBuf d_ctr, d_items, d_over;
    DevBuf d_scratch[3];
    d_ctr.alloc(ctx, 2 * sizeof(unsigned long long));
    d_over.alloc(ctx, sizeof(int32_t));
    // batches: consecutive items of one class within the memory budget
    struct Batch {
        size_t first, last;
        int kind;
        uint64_t elems;
    };
    std::vector<Batch> batches;
    uint64_t kind_max[3] = {0, 0, 0};
    for (size_t s = 0; s < items.size();) {
        size_t e = s;
        uint64_t acc = 0;
        while (e < items.size() && items[e].kind == items[s].kind &&
               (e == s || acc + items[e].bytes <= budget_elems)) {
            acc += items[e].bytes;
            ++e;
        }
        batches.push_back(Batch{s, e, items[s].kind, acc});
        kind_max[items[s].kind] = std::max(kind_max[items[s].kind], acc);
        s = e;
    }
    for (int k = 0; k < 3; ++k)
        if (kind_max[k] > 0) d_scratch[k].alloc(ctx, kind_max[k]);
    if (!p->far_streams_ready) {
        for (int k = 0; k < 3; ++k) GACA_HIP_CHECK(hipStreamCreate(&p->far_streams[k]));
        p->far_streams_ready = true;
    }
    std::vector<FarBlockDev> descs(items.size());
    for (auto &bt : batches) {
        int64_t acc = 0;
        for (size_t k = bt.first; k < bt.last; ++k) {
            FarBlockDev d = items[k].d;
            d.face_off += acc;
            d.uw_off += acc;
            d.fib_off += acc;
            d.gram_off += acc;
            acc += items[k].bytes;
            descs[k] = d;
        }
    }
    d_items.upload(ctx, descs);
    for (int attempt = 0; attempt < 6; ++attempt) {
        h->d_arena.release();
        h->d_fib.release();
        h->d_arena.alloc(ctx, arena_cap * fac_bytes);
        h->d_fib.alloc(ctx, fib_cap * sizeof(double2));
        GACA_HIP_CHECK(hipMemsetAsync(d_ctr.ptr, 0, 2 * sizeof(unsigned long long), st));
        GACA_HIP_CHECK(hipMemsetAsync(d_over.ptr, 0, sizeof(int32_t), st));
        std::vector<hipEvent_t> evs(2 * batches.size() + 4);
        for (auto &e : evs) GACA_HIP_CHECK(hipEventCreate(&e));
        hipEvent_t ev_start = evs[2 * batches.size()];
        GACA_HIP_CHECK(hipEventRecord(ev_start, st));
        for (int k = 0; k < 3; ++k) GACA_HIP_CHECK(hipStreamWaitEvent(p->far_streams[k], ev_start, 0));
        for (size_t bi = 0; bi < batches.size(); ++bi) {
            const Batch &bt = batches[bi];
            hipStream_t fs = p->far_streams[bt.kind];
            GACA_HIP_CHECK(hipEventRecord(evs[2 * bi], fs));
            FarLaunch fl{};
            fl.blocks = d_items.as<FarBlockDev>() + bt.first;
            fl.nb = (int32_t)(bt.last - bt.first);
            fl.kind = bt.kind;
            fl.scratch = d_scratch[bt.kind].ptr;
            fl.mixed = h->prec == GACA_MIXED ? 1 : 0;
            fl.meta = h->d_meta.as<FarMeta>();
            fl.cmeta = h->d_cmeta.as<CrossMeta>();
            fl.cross_off = h->d_cross_off.as<int64_t>();
            fl.arena = h->d_arena.ptr;
            fl.arena_ctr = d_ctr.as<unsigned long long>();
            fl.arena_cap = arena_cap;
            fl.fib_arena = h->d_fib.as<double2>();
            fl.fib_ctr = d_ctr.as<unsigned long long>() + 1;
            fl.fib_cap = fib_cap;
            fl.fib_off = h->d_fib_off.as<int64_t>();
            fl.overflow = d_over.as<int32_t>();
            fl.dense = dense;
            launch_far(h->kernel, p->g, p->f, P, fl, fs);
            GACA_HIP_CHECK(hipGetLastError());
            GACA_HIP_CHECK(hipEventRecord(evs[2 * bi + 1], fs));
        }
        if (attempt == 0) main_work();   // near field on the context stream, concurrently
        for (int k = 0; k < 3; ++k) {
            hipEvent_t done = evs[2 * batches.size() + 1 + k];
            GACA_HIP_CHECK(hipEventRecord(done, p->far_streams[k]));
            GACA_HIP_CHECK(hipStreamWaitEvent(st, done, 0));
        }
        int32_t over = 0;
        unsigned long long ctrs[2];
        GACA_HIP_CHECK(hipMemcpyAsync(&over, d_over.ptr, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        GACA_HIP_CHECK(hipMemcpyAsync(ctrs, d_ctr.ptr, sizeof(ctrs), hipMemcpyDeviceToHost, st));
        GACA_HIP_CHECK(hipStreamSynchronize(st));
        double by_kind[3] = {0, 0, 0}, span = 0.0;
        int nl[3] = {0, 0, 0};
        for (size_t bi = 0; bi < batches.size(); ++bi) {
            float ms = 0.0f, ms_end = 0.0f;
            GACA_HIP_CHECK(hipEventElapsedTime(&ms, evs[2 * bi], evs[2 * bi + 1]));
            GACA_HIP_CHECK(hipEventElapsedTime(&ms_end, ev_start, evs[2 * bi + 1]));
            by_kind[batches[bi].kind] += ms;
            nl[batches[bi].kind] += 1;
            span = std::max(span, (double)ms_end);
        }
        for (auto &e : evs) (void)hipEventDestroy(e);
        for (int k = 0; k < 3; ++k) {
            h->st.ms_far_by_kind[k] = by_kind[k];
            h->st.launches_by_kind[k] = nl[k];
        }
        h->st.ms_far_kernel = span;
        h->st.n_far_launches = (int32_t)batches.size();
        h->st.far_attempts = attempt + 1;
        if (!over) {
            // shrink both arenas to what the build used (offsets are relative to the base)
            compact(ctx, h->d_arena, ctrs[0] * fac_bytes, st);
            compact(ctx, h->d_fib, ctrs[1] * sizeof(double2), st);
            break;
        }
        arena_cap = std::max<uint64_t>(arena_cap * 2, ctrs[0] + 1024);
        fib_cap = std::max<uint64_t>(fib_cap * 2, ctrs[1] + 1024);
        if (attempt == 5) throw Error{GACA_ERR_OOM, "factor arena overflow"};
    }
    GACA_HIP_CHECK(hipMemcpy(h->meta.data(), h->d_meta.ptr, nfar * sizeof(FarMeta), hipMemcpyDeviceToHost));
    GACA_HIP_CHECK(hipMemcpy(h->cmeta.data(), h->d_cmeta.ptr, nfar * rcap * sizeof(CrossMeta), hipMemcpyDeviceToHost));
    GACA_HIP_CHECK(hipMemcpy(h->cross_off.data(), h->d_cross_off.ptr, nfar * rcap * sizeof(int64_t), hipMemcpyDeviceToHost));
    GACA_HIP_CHECK(hipMemcpy(h->fib_off.data(), h->d_fib_off.ptr, nfar * sizeof(int64_t), hipMemcpyDeviceToHost));
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
    // Algorithmic work model (FP64 flops; a complex multiply-add is 8 flops).  Per
    // quadrature-point x frequency evaluation of the single layer: distance 8, sqrt 13
    // (rsq + 2 Newton steps), exp 31 (reduction + degree-13 polynomial + scaling), sincos
    // 36 (Cody-Waite reduction + two polynomials), 1/(4 pi r) 8, weight and complex
    // accumulate 9 -> 105; the double layer adds (1 + s r), r^3 and the numerator: 113.
    const double f_eval = h->kernel == 1 ? 113.0 : 105.0;
    const double qpe = h->kernel == 2 ? 36.0 : 6.0;   // far-rule points per entry
    double macs = 0.0, evals = 0.0;
    double kmacs[3] = {0, 0, 0}, kevals[3] = {0, 0, 0};
    for (int64_t b = 0; b < h->nfar; ++b) {
        const FarMeta &mt = h->meta[b];
        const double m = (double)p->part.far[b][1], n = (double)p->part.far[b][3];
        const int kind = far_kind((int)m, (int)n, h->rcap);
        const double macs0 = macs, evals0 = evals;
        evals += (double)(mt.rank + mt.zero_faces) * m * n * qpe + (double)mt.rank * L * qpe;
        for (int c = 0; c < mt.rank; ++c) {
            const double rho = h->cmeta[b * h->rcap + c].rho;
            macs += c * m * n;                       // residual face: previous crosses
            macs += (m + n) * rho * (rho - 1.0);     // face ACA row/column corrections + Gram
            macs += m * n * rho;                     // dense expansion (pivot search)
            macs += m * n * (c + 1.0);               // <H_l, H_p>
            macs += 2.0 * L * c;                     // fibre correction and fibre dots
        }
        kmacs[kind] += macs - macs0;
        kevals[kind] += evals - evals0;
    }
    for (int k = 0; k < 3; ++k) s.far_flops_by_kind[k] = kevals[k] * f_eval + 8.0 * kmacs[k];
    s.far_kernel_evals = evals;
    s.far_flops = evals * f_eval + 8.0 * macs;
    s.rank_mean = h->nfar ? rsum / h->nfar : 0.0;
    s.face_rank_mean = nfaces > 0 ? frsum / nfaces : 0.0;
    const double eb = h->prec == GACA_FP64 ? 16.0 : 8.0;
    s.bytes_far = (uint64_t)(far_elems * eb + fib_elems * 16.0);
    s.bytes_near = (uint64_t)((double)p->near_elems * eb);
    s.dense_bytes = (double)p->M * (double)p->M * L * eb;
    s.compression = (s.bytes_far + s.bytes_near) / std::max(1.0, s.dense_bytes);
    s.entries_near = (double)p->near_elems;
}

gaca_status gaca_build(gaca_problem *p, gaca_kernel kernel, gaca_hmatrix **out) {
    bool capped = false;
    gaca_status rc = guarded([&] {
        REQUIRE(p && out, "null argument");
        REQUIRE(kernel == GACA_SLP || kernel == GACA_DLP, "bad kernel");
        REQUIRE(!p->synthetic, "build needs a mesh problem");
        REQUIRE(p->opt.precision == GACA_FP64 || p->opt.precision == GACA_MIXED, "bad precision");
        if (p->scheme == GACA_GALERKIN_P0 && kernel != GACA_SLP)
            throw Error{GACA_ERR_UNSUPPORTED, "Galerkin is available for the single layer only"};
        gaca_context *ctx = p->ctx;
        GACA_HIP_CHECK(hipSetDevice(ctx->device));
        auto h = std::make_unique<gaca_hmatrix>();
        h->p = p;
        h->kernel = p->kid(kernel);
        h->prec = p->opt.precision;
        h->rcap = std::max(1, std::min({p->L, p->opt.max_rank3d > 0 ? p->opt.max_rank3d : p->L, 256}));
        const hipStream_t st = ctx->stream;
        const bool mixed = h->prec == GACA_MIXED;
        // near field: FP64 quadrature, stored FP64 or (mixed) FP32
        h->d_near.alloc(ctx, std::max<int64_t>(1, p->near_elems) *
                                 (mixed ? sizeof(float2) : sizeof(double2)));
        hipEvent_t ev[4];
        for (auto &e : ev) GACA_HIP_CHECK(hipEventCreate(&e));
        GACA_HIP_CHECK(hipEventRecord(ev[0], st));
        auto near_work = [&] {
            GACA_HIP_CHECK(hipEventRecord(ev[1], st));
            double2 *n64 = mixed ? nullptr : h->d_near.as<double2>();
            float2 *n32 = mixed ? h->d_near.as<float2>() : nullptr;
            for (int t = 0; t < kNumTiers; ++t) {
                if (p->scheme == GACA_GALERKIN_P0)
                    launch_near_galerkin(t, p->g, p->q, p->f, p->d_pairs[t].as<NearPair>(),
                                         p->npairs[t], p->d_nblocks.as<NearBlockDev>(), n64, n32, st);
                else if (t < 4)
                    launch_near(kernel, t, p->g, p->q, p->f, p->d_pairs[t].as<NearPair>(),
                                p->npairs[t], p->d_nblocks.as<NearBlockDev>(), n64, n32, st);
            }
            GACA_HIP_CHECK(hipGetLastError());
            GACA_HIP_CHECK(hipEventRecord(ev[2], st));
        };
        run_far(h.get(), nullptr, near_work);
        GACA_HIP_CHECK(hipEventRecord(ev[3], st));
        GACA_HIP_CHECK(hipEventSynchronize(ev[3]));
        float ms_near = 0, ms_total = 0;
        GACA_HIP_CHECK(hipEventElapsedTime(&ms_near, ev[1], ev[2]));
        GACA_HIP_CHECK(hipEventElapsedTime(&ms_total, ev[0], ev[3]));
        for (auto &e : ev) (void)hipEventDestroy(e);
        fill_stats(h.get());
        h->st.ms_near = ms_near;
        h->st.ms_near_kernel = ms_near;
        {
            const double le = p->f.L_eval;
            const double ng2 = (double)p->opt.n_galerkin * p->opt.n_galerkin;
            double qp[kNumTiers] = {6.0, 16.0, 64.0, kernel == 0 ? 3.0 * p->opt.n_duffy * p->opt.n_duffy : 0.0, 0.0, 0.0};
            if (p->scheme == GACA_GALERKIN_P0) {
                const double g6[kNumTiers] = {36.0, 256.0, 3.0 * ng2 * ng2, 3.0 * ng2 * ng2,
                                              3.0 * ng2 * ng2, 6.0 * kGalerkinNTheta};
                for (int t = 0; t < kNumTiers; ++t) qp[t] = g6[t];
            }
            double evn = 0.0;
            for (int t = 0; t < kNumTiers; ++t) evn += (double)p->npairs[t] * le * qp[t];
            h->st.near_kernel_evals = evn;
        }
        h->st.ms_far = h->st.ms_far_kernel;
        h->st.ms_total = ms_total;
        capped = h->st.n_capped > 0;
        *out = h.release();
    });
    if (rc == GACA_OK && capped) {
        set_error("rank cap hit in at least one block");
        return GACA_ERR_NOT_CONVERGED;
    }
    return rc;
}

gaca_status gaca_hmatrix_destroy(gaca_hmatrix *h) {
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
        const NearBlockDev &nb = h->p->nblocks[idx];
        const size_t cnt = (size_t)nb.m * nb.n * h->p->L;
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

// ---------------------------------------------------------------------------------------
static void prepare_leaves(gaca_hmatrix *h) {
    if (h->leaf_ready) return;
    gaca_problem *p = h->p;
    gaca_context *ctx = p->ctx;
    const size_t nleaf = p->leaf_r0.size();
    std::vector<std::vector<int32_t>> lf(nleaf), ln(nleaf);
    auto leaves_in = [&](int64_t r0, int64_t m, auto &&fn) {
        auto it = std::lower_bound(p->leaf_r0.begin(), p->leaf_r0.end(), (int32_t)r0);
        for (size_t k = it - p->leaf_r0.begin(); k < nleaf && p->leaf_r0[k] < r0 + m; ++k) fn(k);
    };
    for (int64_t b = 0; b < h->nfar; ++b)
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
    h->d_leaf_r0.upload(ctx, p->leaf_r0);
    h->d_leaf_m.upload(ctx, p->leaf_m);
    h->d_lfp.upload(ctx, fp);
    h->d_lfi.upload(ctx, fi);
    h->d_lnp.upload(ctx, np);
    h->d_lni.upload(ctx, ni);
    h->leaf_ready = true;
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
        if (h->ws_nrhs != nrhs || h->ws_mode != (int)mode || h->ws_dtype != (int)dtype) {
            std::vector<int64_t> zoff(std::max<int64_t>(h->nfar, 1)), toff(std::max<int64_t>(h->nfar, 1)),
                yoff(std::max<int64_t>(h->nfar, 1));
            int64_t zacc = 0, tacc = 0, yacc = 0;
            for (int64_t b = 0; b < h->nfar; ++b) {
                zoff[b] = zacc;
                toff[b] = tacc;
                yoff[b] = yacc;
                yacc += p->part.far[b][1] * (int64_t)nrhs;
                const int64_t sr = h->meta[b].sum_rho;
                zacc += mode == GACA_APPLY_SUM ? sr * nrhs : sr * (int64_t)L * nrhs;
                tacc += mode == GACA_APPLY_SUM ? p->part.far[b][3] * (int64_t)nrhs : 0;
            }
            h->d_zoff.upload(ctx, zoff);
            h->d_toff.upload(ctx, toff);
            h->d_yoff.upload(ctx, yoff);
            h->d_yb.alloc(ctx, std::max<int64_t>(yacc, 1) * xs);
            h->d_z.alloc(ctx, std::max<int64_t>(zacc, 1) * xs);
            h->d_t.alloc(ctx, std::max<int64_t>(tacc, 1) * xs);
            h->d_xp.alloc(ctx, (size_t)L * M * nrhs * xs);
            const int nl = mode == GACA_APPLY_SUM ? 1 : L;
            h->d_yp.alloc(ctx, (size_t)nl * M * nrhs * xs);
            h->ws_nrhs = nrhs;
            h->ws_mode = (int)mode;
            h->ws_dtype = (int)dtype;
        }
        ApplyDev a{};
        a.L = L;
        a.nrhs = nrhs;
        a.M = M;
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
        a.nblocks = p->d_nblocks.as<NearBlockDev>();
        a.near64 = h->prec == GACA_MIXED ? nullptr : h->d_near.as<double2>();
        a.near32 = h->prec == GACA_MIXED ? h->d_near.as<float2>() : nullptr;
        a.nleaf = (int32_t)p->leaf_r0.size();
        a.leaf_r0 = h->d_leaf_r0.as<int32_t>();
        a.leaf_m = h->d_leaf_m.as<int32_t>();
        a.leaf_far_ptr = h->d_lfp.as<int32_t>();
        a.leaf_far_idx = h->d_lfi.as<int32_t>();
        a.leaf_near_ptr = h->d_lnp.as<int32_t>();
        a.leaf_near_idx = h->d_lni.as<int32_t>();
        a.z_off = h->d_zoff.as<int64_t>();
        launch_apply(a, (int)mode, dtype == GACA_C64 ? 1 : 0, X, Y, h->d_xp.ptr, h->d_yp.ptr,
                     h->d_z.ptr, h->d_t.ptr, h->d_toff.as<int64_t>(), h->d_yb.ptr,
                     h->d_yoff.as<int64_t>(), st);
        GACA_HIP_CHECK(hipGetLastError());
    });
}

// ---------------------------------------------------------------------------------------
gaca_status gaca_eval_entries(gaca_problem *p, gaca_kernel kernel, int64_t n, const int32_t *i,
                              const int32_t *j, const int32_t *k, const int32_t *far,
                              double *out) {
    return guarded([&] {
        REQUIRE(p, "null problem");
        REQUIRE(kernel == GACA_SLP || kernel == GACA_DLP, "bad kernel");
        REQUIRE(n >= 0, "n must be >= 0");
        if (n == 0) return;
        REQUIRE(i && j && k && far && out, "null argument");
        REQUIRE(!p->synthetic, "entries need a mesh problem");
        std::vector<int32_t> rows(n), cols(n), ks(n), tiers(n);
        for (int64_t t = 0; t < n; ++t) {
            REQUIRE(i[t] >= 0 && i[t] < p->M && j[t] >= 0 && j[t] < p->M, "element id out of range");
            REQUIRE(k[t] >= 0 && k[t] < p->L, "frequency index out of range");
            rows[t] = (int32_t)p->inv_perm[i[t]];
            cols[t] = (int32_t)p->inv_perm[j[t]];
            ks[t] = k[t];
            if (p->scheme == GACA_GALERKIN_P0)
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
        launch_eval(p->kid(kernel), p->g, p->q, p->f, n, dr.as<int32_t>(), dc.as<int32_t>(), dk.as<int32_t>(),
                    dt.as<int32_t>(), dout.as<double2>(), ctx->stream);
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
        p->ctx = ctx;
        if (opt) p->opt = *opt;
        else options_default(&p->opt);
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
        run_far(h.get(), reinterpret_cast<const double2 *>(dev_tensor), [] {});
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
