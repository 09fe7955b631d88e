// Host runtime behind include/casci.h: argument validation, device memory,
// integral preparation and the Davidson-Liu driver. Every arithmetic step
// on CI vectors runs in the HIP kernels of this directory; the host only
// handles the tiny projected quantities (subspace bookkeeping of at most
// 64 x 64 numbers) and control flow.
#include "casci.h"

#include <algorithm>
#include <array>
#include <atomic>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <cstddef>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "internal.h"

#include <rocblas/rocblas.h>

using namespace casci;

namespace {

// Process-wide cache of large device blocks. A solve allocates ~160 GB of
// basis vectors at CAS(16,16) and frees them at its end; allocating that much
// again after a free cost 1.4-3.8 s per solve (growing with each solve in the
// process), so blocks of at least BLOCK_CACHE_MIN bytes are kept on release
// and handed to later requests of the same or a slightly smaller size. A
// released block is cached only after the device has finished with it (the
// synchronisation hipFree itself performs). At most three quarters of the
// device's memory is held: a block released into a full cache evicts the
// least recently released ones (a later solve repeats the latest one's
// sizes), and an allocation that fails empties the cache of that device and
// is retried. casci_release_cache frees the cached blocks.
constexpr size_t BLOCK_CACHE_MIN = (size_t)64 << 20;
struct BlockCache {
    std::mutex mu;
    std::map<int, std::list<std::pair<size_t, void*>>> free;  // device -> blocks, oldest first
    std::map<int, size_t> held;
};
BlockCache& block_cache()
{
    static BlockCache* c = new BlockCache;  // never destroyed: blocks may outlive static destructors
    return *c;
}
void* cache_take(int dev, size_t b, size_t* got)
{
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto& l = c.free[dev];
    auto best = l.end();
    for (auto it = l.begin(); it != l.end(); ++it)  // smallest block that fits, at most 12.5% larger
        if (it->first >= b && it->first <= b + b / 8 && (best == l.end() || it->first < best->first)) best = it;
    if (best == l.end()) return nullptr;
    void* p = best->second;
    *got = best->first;
    c.held[dev] -= best->first;
    l.erase(best);
    return p;
}
// keeps block p of `bytes` on device dev (current) if it fits under cap after
// evicting the oldest blocks; false: the caller frees it
bool cache_put(int dev, void* p, size_t bytes, size_t cap)
{
    if (bytes > cap) return false;
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto& l = c.free[dev];
    while (!l.empty() && c.held[dev] + bytes > cap) {
        (void)hipFree(l.front().second);
        c.held[dev] -= l.front().first;
        l.pop_front();
    }
    l.emplace_back(bytes, p);
    c.held[dev] += bytes;
    return true;
}
void cache_flush(int dev)
{
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    auto& l = c.free[dev];
    for (auto& kv : l) (void)hipFree(kv.second);
    l.clear();
    c.held[dev] = 0;
}

struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    int dev = -1;
    DBuf() = default;
    DBuf(const DBuf&) = delete;  // one owner per block: a copy would release it twice
    DBuf& operator=(const DBuf&) = delete;
    void swap(DBuf& o)
    {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(dev, o.dev);
    }
    hipError_t ensure(size_t b)
    {
        if (b <= bytes && p) return hipSuccess;
        release();
        if (b == 0) b = 16;
        int d = 0;
        hipError_t e = hipGetDevice(&d);
        if (e != hipSuccess) return e;
        if (b >= BLOCK_CACHE_MIN) {
            size_t got = 0;
            if (void* q = cache_take(d, b, &got)) {
                p = q;
                bytes = got;
                dev = d;
                return hipSuccess;
            }
        }
        e = hipMalloc(&p, b);
        if (e != hipSuccess && b >= BLOCK_CACHE_MIN) {
            (void)hipGetLastError();
            cache_flush(d);
            e = hipMalloc(&p, b);
        }
        if (e != hipSuccess) {
            p = nullptr;
            bytes = 0;
            (void)hipGetLastError();
            return e;
        }
        bytes = b;
        dev = d;
        return hipSuccess;
    }
    void release()
    {
        if (p) {
            bool cached = false;
            if (bytes >= BLOCK_CACHE_MIN) {
                int cur = -1;
                (void)hipGetDevice(&cur);
                if (cur != dev) (void)hipSetDevice(dev);
                size_t fr = 0, tot = 0;
                if (hipDeviceSynchronize() == hipSuccess && hipMemGetInfo(&fr, &tot) == hipSuccess)
                    cached = cache_put(dev, p, bytes, tot / 4 * 3);
                (void)hipGetLastError();
                if (!cached) (void)hipFree(p);
                if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
            } else {
                (void)hipFree(p);
            }
        }
        p = nullptr;
        bytes = 0;
    }
    template <typename T>
    T* as() const
    {
        return reinterpret_cast<T*>(p);
    }
};

struct DeviceGuard {
    int prev = -1;
    bool active = false;
    explicit DeviceGuard(int dev)
    {
        if (dev < 0) return;
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            active = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard()
    {
        if (active) (void)hipSetDevice(prev);
    }
};

int64_t binomial(int n, int k)
{
    if (k < 0 || k > n) return 0;
    long double r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return (int64_t)llroundl(r);
}

}  // namespace

struct casci_ctx {
    int device = -1;
    bool validate_only = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;

    // integrals
    bool has_ints = false;
    int norb_ints = 0;
    std::vector<double> h, eri;
    double ecore = 0.0;

    // strings
    bool has_strings = false;
    int norb = 0, na = 0, nb = 0;
    int64_t Na = 0, Nb = 0, Nd = 0;
    int sa = 0, sb = 0, ra = 0, rb = 0;
    bool ops_sorted = false;  // same-spin operator rows ascending past the diagonal
    std::vector<int64_t> binom;  // (norb+1)^2

    DBuf d_binom, d_astr, d_bstr, d_la_j, d_la_pq, d_lb_j, d_lb_pq;

    // integral-dependent data
    bool prepared = false;
    double prepared_lambda = 0.0;
    DBuf d_h, d_eri, d_fa_col, d_fa_val, d_fb_col, d_fb_val, d_jpq, d_diag;
    DBuf d_fa_c16, d_fa_v32, d_fb_c16, d_fb_v32;  // compact operator copies (< 65536 strings)
    struct Blocks {  // row-blocked form of one same-spin operator (SsBlk)
        DBuf uni, binfo, goff, rbase, gs64, gs32, gsf;
        int64_t nblk = 0;
        int rows = 0;  // rows per block
        bool have = false;
    } blk[2];        // [0]: alpha (and beta when nalpha = nbeta), [1]: beta
    DBuf d_vt_sym, d_pairs_sym, d_vt_full, d_pairs_full, d_vt_s2;
    DBuf d_tg_sym, d_tg_full;  // alpha-beta scatter targets per (beta string, pair row)
    DBuf d_tg16;               // the same (symmetric pairs), 16-bit, in MFMA element order
    struct Reduce {            // target-grouped scatter table (AbReduce) of one pair set
        DBuf tab, tinfo;
        int max_nseg = 0, ldT = 0;
        bool have = false;
    } red_sym, red_full;
    DBuf d_vt_sym_lp[2], d_vt_full_lp[2];  // FP32 and BF16 copies (round to nearest even)
    int M_sym = 0, Mp_sym = 0, M_full = 0, Mp_full = 0;
    bool have_full = false, have_s2 = false;
    // (pq|rs) = (qp|rs) holds (8-fold symmetry): the alpha-beta term can fold
    // the pair rows r <= s; without it (dressed integrals, 4-fold symmetry) it
    // runs over all ordered pairs
    bool eri8 = true;
    bool have_tg_sym = false, have_tg_full = false, have_tg16 = false;

    // workspaces
    DBuf d_t1, d_t2, d_t3, d_vin, d_vout, d_work, d_small, d_clp, d_c32;
    DBuf d_rowmax;  // max_c |C(J, c)| per alpha string: bound of the FP64 alpha-beta fixed-point sums
    // density matrices: pair-excitation rows of a block of alpha strings, their Gram matrix
    DBuf d_rdm_M, d_rdm_G, d_rdm_out;
    rocblas_handle blas = nullptr;

    // learned preconditioner parameters (FP32, MLP_NPARAM values)
    DBuf d_mlp, d_mlp_m, d_mlp_v, d_mlp_g, d_mlp_part, d_mlp_perm, d_mlp_sse, d_mlp_idx;
    bool have_mlp = false;

    // optional per-part timing of sigma builds (HIP events on `stream`)
    bool profiling = false;
    hipEvent_t pev[6] = {};
    double prof[16] = {};

    // state generation: bumped whenever strings, integrals or the prepared
    // operators change (captured sigma graphs of an older generation are stale)
    uint64_t gen = 1;
    // captured sigma builds (graph mode): inputs staged through d_gin/d_gout
    struct Graph {
        int prec, parity;
        double lambda;
        uint64_t gen;
        std::vector<void*> sig;  // device buffers the captured kernels use
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    DBuf d_gin, d_gout;
    // lanes per entry chosen by the autotuner for the FP64 and FP32-input gathers (0: not yet)
    int tune_lpe[2] = {0, 0};
    bool tune_blk[2] = {false, false};  // the tuned width was chosen with the row-blocked form available (or set)
    int tune_ab[2] = {0, 0};  // FP64 alpha-beta layout code per pair set ([0] r <= s, [1] all), 0: untuned

    int fail(int code, const std::string& msg)
    {
        err = msg;
        return code;
    }
};

#define HIPC(expr)                                                                      \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            (void)hipGetLastError();                                                    \
            return ctx->fail(e_ == hipErrorOutOfMemory ? CASCI_E_NOMEM : CASCI_E_DEVICE,  \
                             std::string(#expr) + ": " + hipGetErrorString(e_) +       \
                                 (*launch_reason() ? std::string(" (") + launch_reason() + ")"  \
                                                   : std::string()));                   \
        }                                                                               \
    } while (0)

#define CHECK_RC(expr)          \
    do {                        \
        int rc_ = (expr);       \
        if (rc_ < 0) return rc_; \
    } while (0)

static const char* kValidateOnly = "validate-only context: no device work is launched";

// ---------------------------------------------------------------------------
// static scratch of the allocation-free sigma entry point
// ---------------------------------------------------------------------------
// 64 MiB of device memory per GPU, held until the process ends. Host code never
// passes `scratch` itself to a kernel (in host code the name stands for a
// host-side shadow, not a device address): every use goes through the address
// that hipGetSymbolAddress returned for the device, taken once per device at
// context creation with that device current.
static constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, unsigned char*> g_scratch_addr;  // device -> its copy of `scratch`

static int scratch_setup(int device, std::string* err)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_addr.count(device)) return CASCI_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
        return CASCI_E_DEVICE;
    }
    g_scratch_addr[device] = static_cast<unsigned char*>(p);
    return CASCI_OK;
}

static unsigned char* scratch_addr(int device)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    return it == g_scratch_addr.end() ? nullptr : it->second;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
extern "C" int casci_create(casci_ctx** out, int device, void* hip_stream)
{
    if (!out) return CASCI_E_ARG;
    *out = nullptr;
    casci_ctx* ctx = new (std::nothrow) casci_ctx();
    if (!ctx) return CASCI_E_NOMEM;
    if (device < -1) {
        delete ctx;
        return CASCI_E_ARG;
    }
    if (device == -1) {
        ctx->validate_only = true;
        *out = ctx;
        return CASCI_OK;
    }
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
        (void)hipGetLastError();
        delete ctx;
        return CASCI_E_DEVICE;
    }
    ctx->device = device;
    DeviceGuard g(device);
    {
        std::string why;
        if (scratch_setup(device, &why) != CASCI_OK) {
            delete ctx;
            return CASCI_E_DEVICE;
        }
    }
    if (hip_stream) {
        ctx->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&ctx->stream) != hipSuccess) {
            delete ctx;
            return CASCI_E_DEVICE;
        }
        ctx->own_stream = true;
    }
    *out = ctx;
    return CASCI_OK;
}

extern "C" int casci_release_cache(int device)
{
    std::vector<int> devs;
    {
        BlockCache& c = block_cache();
        std::lock_guard<std::mutex> lk(c.mu);
        for (auto& kv : c.free)
            if (device < 0 || kv.first == device) devs.push_back(kv.first);
    }
    for (int d : devs) {
        DeviceGuard g(d);
        cache_flush(d);
    }
    return CASCI_OK;
}

extern "C" int64_t casci_cached_bytes(int device)
{
    BlockCache& c = block_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    int64_t n = 0;
    for (auto& kv : c.held)
        if (device < 0 || kv.first == device) n += (int64_t)kv.second;
    return n;
}

extern "C" void casci_destroy(casci_ctx* ctx)
{
    if (!ctx) return;
    if (!ctx->validate_only) {
        DeviceGuard g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        DBuf* bufs[] = {&ctx->d_binom, &ctx->d_astr, &ctx->d_bstr, &ctx->d_la_j, &ctx->d_la_pq,
                        &ctx->d_lb_j, &ctx->d_lb_pq, &ctx->d_h, &ctx->d_eri, &ctx->d_fa_col,
                        &ctx->d_fa_val, &ctx->d_fb_col, &ctx->d_fb_val, &ctx->d_jpq, &ctx->d_diag,
                        &ctx->d_vt_sym, &ctx->d_pairs_sym, &ctx->d_vt_full, &ctx->d_pairs_full, &ctx->d_tg_sym, &ctx->d_tg_full, &ctx->d_tg16, &ctx->d_fa_c16, &ctx->d_fa_v32, &ctx->d_fb_c16, &ctx->d_fb_v32,
                        &ctx->red_sym.tab, &ctx->red_sym.tinfo, &ctx->red_full.tab, &ctx->red_full.tinfo,
                        &ctx->d_vt_s2, &ctx->d_t1, &ctx->d_t2, &ctx->d_vin, &ctx->d_vout,
                        &ctx->d_work, &ctx->d_small, &ctx->d_vt_sym_lp[0], &ctx->d_vt_sym_lp[1],
                        &ctx->d_vt_full_lp[0], &ctx->d_vt_full_lp[1], &ctx->d_clp, &ctx->d_c32, &ctx->d_t3,
                        &ctx->d_mlp, &ctx->d_mlp_m, &ctx->d_mlp_v, &ctx->d_mlp_g, &ctx->d_mlp_part,
                        &ctx->d_mlp_perm, &ctx->d_mlp_sse, &ctx->d_mlp_idx, &ctx->d_rowmax,
                        &ctx->d_rdm_M, &ctx->d_rdm_G, &ctx->d_rdm_out};
        if (ctx->blas) (void)rocblas_destroy_handle(ctx->blas);
        for (auto& bl : ctx->blk) {
            for (DBuf* d : {&bl.uni, &bl.binfo, &bl.goff, &bl.rbase, &bl.gs64, &bl.gs32, &bl.gsf}) d->release();
        }
        for (auto& gr : ctx->graphs) (void)hipGraphExecDestroy(gr.exec);
        ctx->graphs.clear();
        ctx->d_gin.release();
        ctx->d_gout.release();
        for (DBuf* b : bufs) b->release();
        for (hipEvent_t& e : ctx->pev)
            if (e) (void)hipEventDestroy(e);
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    }
    delete ctx;
}

extern "C" const char* casci_last_error(const casci_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : "null context";
}

// ---------------------------------------------------------------------------
// integrals
// ---------------------------------------------------------------------------
extern "C" int casci_set_integrals(casci_ctx* ctx, int norb, const double* h, const double* eri,
                                   double e_core, int mem)
{
    if (!ctx) return CASCI_E_ARG;
    if (norb < 1 || norb > 64) return ctx->fail(CASCI_E_ARG, "norb must be in [1, 64]");
    if (!h || !eri) return ctx->fail(CASCI_E_ARG, "h and eri must not be NULL");
    if (mem != CASCI_MEM_HOST && mem != CASCI_MEM_DEVICE) return ctx->fail(CASCI_E_ARG, "bad mem flag");
    if (ctx->has_strings && ctx->norb != norb)
        return ctx->fail(CASCI_E_STATE, "norb differs from the strings already built");
    const size_t n = (size_t)norb, n2 = n * n, n4 = n2 * n2;
    std::vector<double> hh(n2), ee(n4);
    if (mem == CASCI_MEM_DEVICE) {
        if (ctx->validate_only) return ctx->fail(CASCI_E_UNSUPPORTED, kValidateOnly);
        DeviceGuard g(ctx->device);
        HIPC(hipMemcpyAsync(hh.data(), h, n2 * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipMemcpyAsync(ee.data(), eri, n4 * 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
    } else {
        std::memcpy(hh.data(), h, n2 * 8);
        std::memcpy(ee.data(), eri, n4 * 8);
    }
    if (!std::isfinite(e_core)) return ctx->fail(CASCI_E_NONFINITE, "e_core is not finite");
    double hmax = 0.0, emax = 0.0;
    for (double v : hh) {
        if (!std::isfinite(v)) return ctx->fail(CASCI_E_NONFINITE, "h has a non-finite entry");
        hmax = std::max(hmax, std::fabs(v));
    }
    for (double v : ee) {
        if (!std::isfinite(v)) return ctx->fail(CASCI_E_NONFINITE, "eri has a non-finite entry");
        emax = std::max(emax, std::fabs(v));
    }
    const double th = 1e-12 * std::max(1.0, hmax), te = 1e-12 * std::max(1.0, emax);
    for (size_t p = 0; p < n; ++p)
        for (size_t q = 0; q < n; ++q)
            if (std::fabs(hh[p * n + q] - hh[q * n + p]) > th)
                return ctx->fail(CASCI_E_ARG, "h is not symmetric");
    auto E = [&](size_t p, size_t q, size_t r, size_t s) { return ee[((p * n + q) * n + r) * n + s]; };
    // A Hermitian Hamiltonian needs (pq|rs) = (qp|sr) and (pq|rs) = (rs|pq)
    // (4-fold); ordinary integrals of real orbitals also have (pq|rs) = (qp|rs)
    // (8-fold), dressed (similarity-transformed) ones need not
    bool sym8 = true;
    for (size_t p = 0; p < n; ++p)
        for (size_t q = 0; q < n; ++q)
            for (size_t r = 0; r < n; ++r)
                for (size_t s = 0; s < n; ++s) {
                    double v = E(p, q, r, s);
                    if (std::fabs(v - E(q, p, s, r)) > te || std::fabs(v - E(r, s, p, q)) > te)
                        return ctx->fail(CASCI_E_ARG,
                                         "eri lacks the symmetry (pq|rs) = (qp|sr) = (rs|pq) of a Hermitian H");
                    if (std::fabs(v - E(q, p, r, s)) > te) sym8 = false;
                }
    ctx->h.swap(hh);
    ctx->eri.swap(ee);
    ctx->eri8 = sym8;
    ctx->ecore = e_core;
    ctx->norb_ints = norb;
    ctx->has_ints = true;
    ctx->prepared = false;
    ctx->have_full = ctx->have_s2 = false;
    ctx->have_tg_sym = ctx->have_tg_full = ctx->have_tg16 = false;
    ctx->blk[0].have = ctx->blk[1].have = false;
    ctx->red_sym.have = ctx->red_full.have = false;
    ++ctx->gen;
    return CASCI_OK;
}

// ---------------------------------------------------------------------------
// strings
// ---------------------------------------------------------------------------
static int64_t predicted_bytes(int64_t Na, int64_t Nb, int sa, int sb, int ra, int rb)
{
    const int64_t Nd = Na * Nb;
    int64_t b = 8 * (Na + Nb) + 6 * (Na * (int64_t)sa + Nb * (int64_t)sb);
    b += 12 * (Na * (int64_t)ra + Nb * (int64_t)rb);
    b += 8 * Nd * 5;  // diagonal, two sigma temporaries, one C/sigma pair
    return b;
}

extern "C" int casci_build_strings(casci_ctx* ctx, int nalpha, int nbeta, int norb)
{
    if (!ctx) return CASCI_E_ARG;
    if (norb < 1 || norb > 64) return ctx->fail(CASCI_E_ARG, "norb must be in [1, 64]");
    if (nalpha < 0 || nbeta < 0 || nalpha > norb || nbeta > norb)
        return ctx->fail(CASCI_E_ARG, "need 0 <= nalpha, nbeta <= norb");
    if (ctx->has_ints && ctx->norb_ints != norb)
        return ctx->fail(CASCI_E_STATE, "norb differs from the integrals already set");
    const int64_t Na = binomial(norb, nalpha), Nb = binomial(norb, nbeta);
    if (Na >= (1LL << 31) || Nb >= (1LL << 31))
        return ctx->fail(CASCI_E_NOMEM, "more than 2^31 strings per spin");
    if (Na > 0 && Nb > (int64_t)9e18 / Na) return ctx->fail(CASCI_E_NOMEM, "determinant count overflows");
    const int sa = nalpha * (norb - nalpha + 1), sb = nbeta * (norb - nbeta + 1);
    auto rcount = [&](int ne) {
        return (int)(1 + ne * (norb - ne) + binomial(ne, 2) * binomial(norb - ne, 2));
    };
    const int ra = rcount(nalpha), rb = rcount(nbeta);
    const int64_t need = predicted_bytes(Na, Nb, sa, sb, ra, rb);
    if (need > (1LL << 40)) return ctx->fail(CASCI_E_NOMEM, "predicted device memory exceeds 1 TiB");
    std::vector<int64_t> binom((size_t)(norb + 1) * (norb + 1));
    for (int p = 0; p <= norb; ++p)
        for (int k = 0; k <= norb; ++k) binom[(size_t)p * (norb + 1) + k] = binomial(p, k);

    if (!ctx->validate_only) {
        DeviceGuard g(ctx->device);
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && (size_t)need > fr)
            return ctx->fail(CASCI_E_NOMEM, "predicted device memory exceeds free memory");
        (void)hipGetLastError();
        casci_ctx tmp;  // build into fresh buffers so a failure leaves no partial state
        HIPC(tmp.d_binom.ensure(binom.size() * 8));
        HIPC(tmp.d_astr.ensure(Na * 8));
        HIPC(tmp.d_bstr.ensure(Nb * 8));
        HIPC(tmp.d_la_j.ensure(Na * (size_t)sa * 4));
        HIPC(tmp.d_la_pq.ensure(Na * (size_t)sa * 2));
        HIPC(tmp.d_lb_j.ensure(Nb * (size_t)sb * 4));
        HIPC(tmp.d_lb_pq.ensure(Nb * (size_t)sb * 2));
        HIPC(hipMemcpyAsync(tmp.d_binom.p, binom.data(), binom.size() * 8, hipMemcpyHostToDevice,
                            ctx->stream));
        HIPC(launch_build_strings(norb, nalpha, Na, tmp.d_binom.as<int64_t>(), tmp.d_astr.as<uint64_t>(),
                                  ctx->stream));
        HIPC(launch_build_strings(norb, nbeta, Nb, tmp.d_binom.as<int64_t>(), tmp.d_bstr.as<uint64_t>(),
                                  ctx->stream));
        HIPC(launch_single_lists(norb, nalpha, Na, tmp.d_astr.as<uint64_t>(), tmp.d_binom.as<int64_t>(),
                                 sa, tmp.d_la_j.as<int32_t>(), tmp.d_la_pq.as<uint16_t>(), ctx->stream));
        HIPC(launch_single_lists(norb, nbeta, Nb, tmp.d_bstr.as<uint64_t>(), tmp.d_binom.as<int64_t>(),
                                 sb, tmp.d_lb_j.as<int32_t>(), tmp.d_lb_pq.as<uint16_t>(), ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
        ctx->d_binom.swap(tmp.d_binom);
        ctx->d_astr.swap(tmp.d_astr);
        ctx->d_bstr.swap(tmp.d_bstr);
        ctx->d_la_j.swap(tmp.d_la_j);
        ctx->d_la_pq.swap(tmp.d_la_pq);
        ctx->d_lb_j.swap(tmp.d_lb_j);
        ctx->d_lb_pq.swap(tmp.d_lb_pq);
        DBuf* old[] = {&tmp.d_binom, &tmp.d_astr, &tmp.d_bstr, &tmp.d_la_j,
                       &tmp.d_la_pq, &tmp.d_lb_j, &tmp.d_lb_pq};
        for (DBuf* b : old) b->release();
    }
    ctx->binom.swap(binom);
    ctx->norb = norb;
    ctx->na = nalpha;
    ctx->nb = nbeta;
    ctx->Na = Na;
    ctx->Nb = Nb;
    ctx->Nd = Na * Nb;
    ctx->sa = sa;
    ctx->sb = sb;
    ctx->ra = ra;
    ctx->rb = rb;
    ctx->has_strings = true;
    ctx->tune_lpe[0] = ctx->tune_lpe[1] = 0;
    ctx->tune_blk[0] = ctx->tune_blk[1] = false;
    ctx->tune_ab[0] = ctx->tune_ab[1] = 0;
    ctx->prepared = false;
    ctx->have_full = ctx->have_s2 = false;
    ctx->have_tg_sym = ctx->have_tg_full = ctx->have_tg16 = false;
    ctx->blk[0].have = ctx->blk[1].have = false;
    ctx->red_sym.have = ctx->red_full.have = false;
    ++ctx->gen;
    return CASCI_OK;
}

extern "C" int casci_get_dims(const casci_ctx* ctx, int64_t* dims)
{
    if (!ctx || !dims) return CASCI_E_ARG;
    if (!ctx->has_strings) return CASCI_E_STATE;
    dims[0] = ctx->Na;
    dims[1] = ctx->Nb;
    dims[2] = ctx->Nd;
    dims[3] = ctx->sa;
    dims[4] = ctx->sb;
    dims[5] = ctx->ra;
    dims[6] = ctx->rb;
    dims[7] = ctx->norb;
    return CASCI_OK;
}

static int need_device(casci_ctx* ctx)
{
    if (ctx->validate_only) return ctx->fail(CASCI_E_UNSUPPORTED, kValidateOnly);
    return CASCI_OK;
}

extern "C" int casci_get_strings(casci_ctx* ctx, int spin, uint64_t* out)
{
    if (!ctx) return CASCI_E_ARG;
    if (spin != 0 && spin != 1) return ctx->fail(CASCI_E_ARG, "spin must be 0 or 1");
    if (!out) return ctx->fail(CASCI_E_ARG, "out is NULL");
    if (!ctx->has_strings) return ctx->fail(CASCI_E_STATE, "build_strings first");
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    const DBuf& b = spin ? ctx->d_bstr : ctx->d_astr;
    const int64_t N = spin ? ctx->Nb : ctx->Na;
    HIPC(hipMemcpyAsync(out, b.p, N * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return CASCI_OK;
}

extern "C" int casci_get_single_list(casci_ctx* ctx, int spin, int32_t* J, int8_t* sign, uint8_t* p,
                                     uint8_t* q)
{
    if (!ctx) return CASCI_E_ARG;
    if (spin != 0 && spin != 1) return ctx->fail(CASCI_E_ARG, "spin must be 0 or 1");
    if (!ctx->has_strings) return ctx->fail(CASCI_E_STATE, "build_strings first");
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    const int64_t N = spin ? ctx->Nb : ctx->Na;
    const int s = spin ? ctx->sb : ctx->sa;
    const size_t cnt = (size_t)N * s;
    std::vector<int32_t> lj(cnt);
    std::vector<uint16_t> lpq(cnt);
    if (cnt) {
        HIPC(hipMemcpyAsync(lj.data(), (spin ? ctx->d_lb_j : ctx->d_la_j).p, cnt * 4,
                            hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipMemcpyAsync(lpq.data(), (spin ? ctx->d_lb_pq : ctx->d_la_pq).p, cnt * 2,
                            hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
    }
    for (size_t i = 0; i < cnt; ++i) {
        if (J) J[i] = l1_index(lj[i]);
        if (sign) sign[i] = (int8_t)l1_sign(lj[i]);
        if (p) p[i] = (uint8_t)(lpq[i] & 0xff);
        if (q) q[i] = (uint8_t)(lpq[i] >> 8);
    }
    return CASCI_OK;
}

// ---------------------------------------------------------------------------
// integral-dependent preparation
// ---------------------------------------------------------------------------
static void pair_tables(int n, bool full, std::vector<uint16_t>& pairs, int& M, int& Mp)
{
    pairs.clear();
    for (int r = 0; r < n; ++r)
        for (int s = full ? 0 : r; s < n; ++s) pairs.push_back((uint16_t)(r | (s << 8)));
    M = (int)pairs.size();
    Mp = (M + 15) / 16 * 16;
    pairs.resize(Mp, 0xffff);
}

// Vt[pq][m] = (pq|r_m s_m) + coefficient of the S^2 penalty:
// lambda * S^2 contains -lambda sum_pq E^a_qp E^b_pq, i.e. -lambda on
// (alpha pair (p,q), beta pair (r,s)) whenever p = s and q = r.
static void build_vt(const casci_ctx* ctx, const std::vector<uint16_t>& pairs, int M, int Mp,
                     double eri_scale, double penalty, std::vector<double>& vt)
{
    const int n = ctx->norb;
    vt.assign((size_t)n * n * Mp, 0.0);
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q)
            for (int m = 0; m < M; ++m) {
                const int r = pairs[m] & 0xff, s = pairs[m] >> 8;
                double v = eri_scale * ctx->eri[(((size_t)p * n + q) * n + r) * n + s];
                if (p == s && q == r) v -= penalty;
                vt[((size_t)p * n + q) * Mp + m] = v;
            }
}

// FP64 -> BF16 with round-to-nearest-even. The FP64 -> FP32 step is itself
// RNE and can only mislead the second rounding when it lands exactly on a
// BF16 tie; then the side of the tie is taken from the FP64 value.
static uint16_t bf16_rne(double x)
{
    const float f = (float)x;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
    if ((u & 0xffffu) == 0x8000u) {
        const double back = (double)f;
        if (std::fabs(x) > std::fabs(back)) u += 1;       // above the tie in magnitude
        else if (std::fabs(x) < std::fabs(back)) u -= 1;  // below it
    }
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

static int upload_lowp(casci_ctx* ctx, const std::vector<double>& vt, DBuf* lp)
{
    std::vector<float> f(vt.size());
    std::vector<uint16_t> b(vt.size());
    for (size_t i = 0; i < vt.size(); ++i) {
        f[i] = (float)vt[i];
        b[i] = bf16_rne(vt[i]);
    }
    HIPC(lp[0].ensure(f.size() * 4));
    HIPC(lp[1].ensure(b.size() * 2));
    HIPC(hipMemcpyAsync(lp[0].p, f.data(), f.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipMemcpyAsync(lp[1].p, b.data(), b.size() * 2, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return CASCI_OK;
}

static int ensure_prepared(casci_ctx* ctx, double lambda)
{
    if (!ctx->has_ints) return ctx->fail(CASCI_E_STATE, "set_integrals first");
    if (!ctx->has_strings) return ctx->fail(CASCI_E_STATE, "build_strings first");
    if (ctx->norb != ctx->norb_ints) return ctx->fail(CASCI_E_STATE, "norb mismatch");
    CHECK_RC(need_device(ctx));
    const int n = ctx->norb;
    hipStream_t st = ctx->stream;
    if (!ctx->prepared) {
        HIPC(ctx->d_h.ensure((size_t)n * n * 8));
        HIPC(ctx->d_eri.ensure((size_t)n * n * n * n * 8));
        HIPC(hipMemcpyAsync(ctx->d_h.p, ctx->h.data(), (size_t)n * n * 8, hipMemcpyHostToDevice, st));
        HIPC(hipMemcpyAsync(ctx->d_eri.p, ctx->eri.data(), (size_t)n * n * n * n * 8,
                            hipMemcpyHostToDevice, st));
        HIPC(ctx->d_fa_col.ensure((size_t)ctx->Na * ctx->ra * 4));
        HIPC(ctx->d_fa_val.ensure((size_t)ctx->Na * ctx->ra * 8));
        HIPC(launch_same_spin_operator(n, ctx->na, ctx->Na, ctx->d_astr.as<uint64_t>(),
                                       ctx->d_binom.as<int64_t>(), ctx->d_h.as<double>(),
                                       ctx->d_eri.as<double>(), ctx->ra, ctx->d_fa_col.as<int32_t>(),
                                       ctx->d_fa_val.as<double>(), st));
        // rows in ascending column order past the diagonal: the canonical
        // summation order of every gather, and what the row-blocked form needs
        const auto sortable = [](int r) { return r - 1 <= sort_ss_rows_max(); };
        ctx->ops_sorted = sortable(ctx->ra) && (ctx->nb == ctx->na || sortable(ctx->rb));
        if (ctx->ops_sorted)
            HIPC(launch_sort_ss_rows(ctx->Na, ctx->ra, ctx->d_fa_col.as<int32_t>(), ctx->d_fa_val.as<double>(), st));
        if (ctx->nb != ctx->na) {
            HIPC(ctx->d_fb_col.ensure((size_t)ctx->Nb * ctx->rb * 4));
            HIPC(ctx->d_fb_val.ensure((size_t)ctx->Nb * ctx->rb * 8));
            HIPC(launch_same_spin_operator(n, ctx->nb, ctx->Nb, ctx->d_bstr.as<uint64_t>(),
                                           ctx->d_binom.as<int64_t>(), ctx->d_h.as<double>(),
                                           ctx->d_eri.as<double>(), ctx->rb,
                                           ctx->d_fb_col.as<int32_t>(), ctx->d_fb_val.as<double>(), st));
            if (ctx->ops_sorted)
                HIPC(launch_sort_ss_rows(ctx->Nb, ctx->rb, ctx->d_fb_col.as<int32_t>(), ctx->d_fb_val.as<double>(),
                                         st));
        } else {
            ctx->d_fb_col.release();
            ctx->d_fb_val.release();
        }
        // compact copies for the gathers: 16-bit columns, FP32 values
        if (ctx->Na < 65536) {
            HIPC(ctx->d_fa_c16.ensure((size_t)ctx->Na * ctx->ra * 2));
            HIPC(ctx->d_fa_v32.ensure((size_t)ctx->Na * ctx->ra * 4));
            HIPC(launch_compact_op(ctx->d_fa_col.as<int32_t>(), ctx->d_fa_val.as<double>(), ctx->Na * ctx->ra,
                                   ctx->d_fa_c16.as<uint16_t>(), ctx->d_fa_v32.as<float>(), st));
        } else {
            ctx->d_fa_c16.release();
            ctx->d_fa_v32.release();
        }
        if (ctx->nb != ctx->na && ctx->Nb < 65536) {
            HIPC(ctx->d_fb_c16.ensure((size_t)ctx->Nb * ctx->rb * 2));
            HIPC(ctx->d_fb_v32.ensure((size_t)ctx->Nb * ctx->rb * 4));
            HIPC(launch_compact_op(ctx->d_fb_col.as<int32_t>(), ctx->d_fb_val.as<double>(), ctx->Nb * ctx->rb,
                                   ctx->d_fb_c16.as<uint16_t>(), ctx->d_fb_v32.as<float>(), st));
        } else {
            ctx->d_fb_c16.release();
            ctx->d_fb_v32.release();
        }
        std::vector<double> jpq((size_t)n * n);
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) jpq[p * n + q] = ctx->eri[(((size_t)p * n + p) * n + q) * n + q];
        HIPC(ctx->d_jpq.ensure(jpq.size() * 8));
        HIPC(hipMemcpyAsync(ctx->d_jpq.p, jpq.data(), jpq.size() * 8, hipMemcpyHostToDevice, st));
        std::vector<uint16_t> pairs;
        std::vector<double> vt;
        pair_tables(n, false, pairs, ctx->M_sym, ctx->Mp_sym);
        build_vt(ctx, pairs, ctx->M_sym, ctx->Mp_sym, 1.0, 0.0, vt);
        HIPC(ctx->d_pairs_sym.ensure(pairs.size() * 2));
        HIPC(ctx->d_vt_sym.ensure(vt.size() * 8));
        HIPC(hipMemcpyAsync(ctx->d_pairs_sym.p, pairs.data(), pairs.size() * 2, hipMemcpyHostToDevice, st));
        HIPC(hipMemcpyAsync(ctx->d_vt_sym.p, vt.data(), vt.size() * 8, hipMemcpyHostToDevice, st));
        // pageable host sources: finish before the vectors go out of scope
        HIPC(hipStreamSynchronize(st));
        CHECK_RC(upload_lowp(ctx, vt, ctx->d_vt_sym_lp));
        ctx->prepared = true;
        ctx->have_full = false;
        ctx->have_tg_sym = ctx->have_tg_full = ctx->have_tg16 = false;
        ctx->red_sym.have = ctx->red_full.have = false;
        ++ctx->gen;
        ctx->prepared_lambda = std::nan("");
    }
    if (!(ctx->prepared_lambda == lambda)) {
        HIPC(ctx->d_diag.ensure((size_t)ctx->Nd * 8));
        const bool same = ctx->nb == ctx->na;
        HIPC(launch_diagonal(n, ctx->Na, ctx->Nb, ctx->d_astr.as<uint64_t>(), ctx->d_bstr.as<uint64_t>(),
                             ctx->d_fa_val.as<double>(), ctx->ra,
                             (same ? ctx->d_fa_val : ctx->d_fb_val).as<double>(), ctx->rb,
                             ctx->d_jpq.as<double>(), ctx->ecore, lambda, ctx->d_diag.as<double>(), st));
        // all ordered pairs: with the S^2 penalty (not symmetric in rs) or
        // integrals without the 8-fold symmetry
        if (lambda != 0.0 || !ctx->eri8) {
            std::vector<uint16_t> pairs;
            std::vector<double> vt;
            pair_tables(n, true, pairs, ctx->M_full, ctx->Mp_full);
            build_vt(ctx, pairs, ctx->M_full, ctx->Mp_full, 1.0, lambda, vt);
            HIPC(ctx->d_pairs_full.ensure(pairs.size() * 2));
            HIPC(ctx->d_vt_full.ensure(vt.size() * 8));
            HIPC(hipMemcpyAsync(ctx->d_pairs_full.p, pairs.data(), pairs.size() * 2,
                                hipMemcpyHostToDevice, st));
            HIPC(hipMemcpyAsync(ctx->d_vt_full.p, vt.data(), vt.size() * 8, hipMemcpyHostToDevice, st));
            HIPC(hipStreamSynchronize(st));
            CHECK_RC(upload_lowp(ctx, vt, ctx->d_vt_full_lp));
            ctx->have_full = true;
        }
        ctx->prepared_lambda = lambda;
        ++ctx->gen;
    }
    return CASCI_OK;
}

static AbParams ab_params(const casci_ctx* ctx, bool full)
{
    AbParams p;
    p.n = ctx->norb;
    p.nb = ctx->nb;
    p.Na = ctx->Na;
    p.Nb = ctx->Nb;
    p.sa = ctx->sa;
    p.M = full ? ctx->M_full : ctx->M_sym;
    p.Mp = full ? ctx->Mp_full : ctx->Mp_sym;
    p.full = full ? 1 : 0;
    p.la_j = ctx->d_la_j.as<int32_t>();
    p.la_pq = ctx->d_la_pq.as<uint16_t>();
    p.bstr = ctx->d_bstr.as<uint64_t>();
    p.lb_j = ctx->d_lb_j.as<int32_t>();
    p.sb = ctx->sb;
    p.overwrite = 0;
    p.pairs = (full ? ctx->d_pairs_full : ctx->d_pairs_sym).as<uint16_t>();
    p.tg = (full ? ctx->d_tg_full : ctx->d_tg_sym).as<int32_t>();
    return p;
}

// scatter-target table of the pair set (needs the strings, lists and pairs on device)
static int ensure_targets(casci_ctx* ctx, bool full, bool may_alloc = true)
{
    bool& have = full ? ctx->have_tg_full : ctx->have_tg_sym;
    if (have) return CASCI_OK;
    if (!may_alloc)
        return ctx->fail(CASCI_E_STATE, "alpha-beta scatter targets not built: run casci_sigma once first");
    DBuf& tg = full ? ctx->d_tg_full : ctx->d_tg_sym;
    AbParams p = ab_params(ctx, full);
    HIPC(tg.ensure((size_t)ctx->Nb * p.Mp * 4));
    p.tg = tg.as<int32_t>();
    HIPC(launch_ab_targets(p, tg.as<int32_t>(), ctx->stream));
    have = true;
    return CASCI_OK;
}

// 16-bit targets of the symmetric pair set in MFMA element order (the BF16
// fixed-point kernel), converted from the 32-bit table
static int ensure_tg16(casci_ctx* ctx, bool may_alloc = true)
{
    if (ctx->have_tg16) return CASCI_OK;
    if (!may_alloc) return ctx->fail(CASCI_E_STATE, "16-bit scatter targets not built: run casci_sigma once first");
    CHECK_RC(ensure_targets(ctx, false));
    HIPC(ctx->d_tg16.ensure((size_t)tg16_entries(ctx->Nb, ctx->Mp_sym) * 2));
    HIPC(launch_tg16(ctx->d_tg_sym.as<int32_t>(), ctx->Nb, ctx->Mp_sym, ctx->d_tg16.as<uint16_t>(), ctx->stream));
    ctx->have_tg16 = true;
    return CASCI_OK;
}

// Target-grouped table of the low-precision alpha-beta kernel (layout in
// internal.h, AbReduce), built on the host from the target table.
static int ensure_reduce(casci_ctx* ctx, bool full, AbReduce* out, bool may_alloc = true)
{
    casci_ctx::Reduce& R = full ? ctx->red_full : ctx->red_sym;
    if (!R.have && !may_alloc)
        return ctx->fail(CASCI_E_STATE, "alpha-beta reduction table not built: run casci_sigma once first");
    if (!R.have) {
        CHECK_RC(ensure_targets(ctx, full));
        const int Mp = full ? ctx->Mp_full : ctx->Mp_sym;
        const int64_t Nb = ctx->Nb;
        const int TN = 64;
        const int ldT = Mp + 4;
        const int zslot = TN * ldT;
        if (zslot + 1 > 0x7fff)
            return ctx->fail(CASCI_E_UNSUPPORTED, "alpha-beta: too many pair rows for the low-precision table");
        if (Nb >= 0xffff)
            return ctx->fail(CASCI_E_UNSUPPORTED, "alpha-beta: more than 65534 beta strings for the low-precision table");
        std::vector<int32_t> tg((size_t)Nb * Mp);
        HIPC(hipMemcpyAsync(tg.data(), (full ? ctx->d_tg_full : ctx->d_tg_sym).p, tg.size() * 4,
                            hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
        const int64_t ntiles = (Nb + TN - 1) / TN;
        const int W = abl_waves(Mp);
        std::vector<uint32_t> words;
        std::vector<int32_t> tinfo((size_t)ntiles * 2);
        std::vector<std::pair<int32_t, uint16_t>> con;
        struct Group {
            int32_t target;
            int begin, count;
        };
        std::vector<Group> grp;
        std::vector<uint16_t> off;
        int max_nseg = 0;
        for (int64_t t = 0; t < ntiles; ++t) {
            con.clear();
            for (int jl = 0; jl < TN && t * TN + jl < Nb; ++jl)
                for (int m = 0; m < Mp; ++m) {
                    const int32_t e = tg[(size_t)(t * TN + jl) * Mp + m];
                    if (e == INT32_MIN) continue;
                    con.push_back({l1_index(e), (uint16_t)((jl * ldT + m) | (e < 0 ? 0x8000 : 0))});
                }
            std::stable_sort(con.begin(), con.end(),
                             [](const std::pair<int32_t, uint16_t>& a, const std::pair<int32_t, uint16_t>& b) {
                                 return a.first < b.first;
                             });
            grp.clear();
            for (size_t i = 0; i < con.size();) {
                size_t j = i;
                while (j < con.size() && con[j].first == con[i].first) ++j;
                grp.push_back({con[i].first, (int)i, (int)(j - i)});
                i = j;
            }
            std::stable_sort(grp.begin(), grp.end(), [](const Group& a, const Group& b) { return a.count > b.count; });
            // chunks of 64 groups, largest first; blocks of 4 contributions
            const int nreal = (int)((grp.size() + 63) / 64);
            std::vector<int> cblocks(nreal);
            for (int q = 0; q < nreal; ++q) cblocks[q] = (grp[(size_t)q * 64].count + 3) / 4;
            // longest-first assignment to the least loaded wave; the chunks of
            // wave w are stored contiguously, wave by wave
            std::vector<std::vector<int>> per_wave(W);
            std::vector<int64_t> load(W, 0);
            for (int q = 0; q < nreal; ++q) {
                const int w = (int)(std::min_element(load.begin(), load.end()) - load.begin());
                per_wave[w].push_back(q);
                load[w] += cblocks[q] + 1;
            }
            std::vector<int> order;
            std::vector<uint16_t> wb(((size_t)W + 1 + 7) / 8 * 8, 0);
            for (int w = 0; w < W; ++w) {
                order.insert(order.end(), per_wave[w].begin(), per_wave[w].end());
                wb[w + 1] = (uint16_t)order.size();
            }
            const int nch = (int)order.size();
            const int dsegs = (nch + 3) / 4;
            const size_t seg0 = words.size() / 4;
            for (size_t i = 0; i < wb.size(); i += 2) words.push_back((uint32_t)wb[i] | ((uint32_t)wb[i + 1] << 16));
            std::vector<uint32_t> desc((size_t)dsegs * 4, 0u);
            int blocks = 0;
            for (int q = 0; q < nch; ++q) {
                const int nb = cblocks[order[q]];
                if (nb >= 4096 || blocks + nb >= (1 << 20))
                    return ctx->fail(CASCI_E_UNSUPPORTED, "alpha-beta: scatter table tile too large");
                desc[q] = (uint32_t)blocks | ((uint32_t)nb << 20);
                blocks += nb;
            }
            words.insert(words.end(), desc.begin(), desc.end());
            for (int q = 0; q < nch; ++q)
                for (int lane = 0; lane < 64; lane += 2) {
                    uint32_t pr = 0;
                    for (int h = 0; h < 2; ++h) {
                        const size_t g = (size_t)order[q] * 64 + lane + h;
                        const uint32_t v = g < grp.size() ? (uint32_t)grp[g].target : 0xffffu;
                        pr |= v << (16 * h);
                    }
                    words.push_back(pr);
                }
            off.assign((size_t)blocks * 256, (uint16_t)zslot);
            for (int q = 0; q < nch; ++q) {
                const int cb = (int)(desc[q] & 0xfffff);
                for (int lane = 0; lane < 64; ++lane) {
                    const size_t g = (size_t)order[q] * 64 + lane;
                    if (g >= grp.size()) continue;
                    for (int c = 0; c < grp[g].count; ++c)
                        off[((size_t)(cb + c / 4) * 64 + lane) * 4 + c % 4] = con[grp[g].begin + c].second;
                }
            }
            for (size_t i = 0; i < off.size(); i += 2) words.push_back((uint32_t)off[i] | ((uint32_t)off[i + 1] << 16));
            const size_t nseg = words.size() / 4 - seg0;
            if (seg0 > 0x7fffffff || nseg >= (1u << 20))
                return ctx->fail(CASCI_E_UNSUPPORTED, "alpha-beta: scatter table too large");
            tinfo[(size_t)t * 2] = (int32_t)seg0;
            tinfo[(size_t)t * 2 + 1] = (int32_t)(nseg | ((size_t)nch << 20));
            max_nseg = std::max(max_nseg, (int)nseg);
        }
        if (words.empty()) words.assign(4, 0u);
        HIPC(R.tab.ensure(words.size() * 4));
        HIPC(R.tinfo.ensure(tinfo.size() * 4 + 8));
        HIPC(hipMemcpyAsync(R.tab.p, words.data(), words.size() * 4, hipMemcpyHostToDevice, ctx->stream));
        HIPC(hipMemcpyAsync(R.tinfo.p, tinfo.data(), tinfo.size() * 4, hipMemcpyHostToDevice, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
        R.max_nseg = max_nseg;
        R.ldT = ldT;
        R.have = true;
    }
    out->tab = R.tab.as<uint4>();
    out->tinfo = R.tinfo.as<int2>();
    out->max_nseg = R.max_nseg;
    out->ldT = R.ldT;
    return CASCI_OK;
}

// The same-spin operator of one spin (1: beta; the alpha one when nalpha = nbeta)
// with its compact copies when they exist.
static SsOp ss_op(const casci_ctx* ctx, int spin)
{
    const bool b = spin == 1 && ctx->nb != ctx->na;
    SsOp op;
    op.col = (b ? ctx->d_fb_col : ctx->d_fa_col).as<int32_t>();
    op.val = (b ? ctx->d_fb_val : ctx->d_fa_val).as<double>();
    op.col16 = (b ? ctx->d_fb_c16 : ctx->d_fa_c16).as<uint16_t>();
    op.val32 = (b ? ctx->d_fb_v32 : ctx->d_fa_v32).as<float>();
    op.r = spin == 1 ? ctx->rb : ctx->ra;
    const casci_ctx::Blocks& bl = ctx->blk[b ? 1 : 0];
    if (bl.have) {
        op.blk.uni = bl.uni.as<uint16_t>();
        op.blk.binfo = bl.binfo.as<int4>();
        op.blk.goff = bl.goff.as<uint16_t>();
        op.blk.rbase = bl.rbase.as<int32_t>();
        op.blk.gs64 = bl.gs64.as<SsGroup>();
        op.blk.gs32 = bl.gs32.as<SsGroup>();
        op.blk.gsf = bl.gsf.as<SsGroupF>();
        op.blk.ch = SS_BLK_CH;
        op.blk.nblk = bl.nblk;
        op.blk.rows = bl.rows;
    }
    return op;
}

// Row-blocked form of a same-spin operator for the SS_BLOCKED gather: rows in
// blocks of 32 (or 16), the sorted union of the columns of each block, and per
// row its entries 1..r-1 (ascending columns) as groups of four aligned to the
// entry index, split by chunks of SS_BLK_CH union rows: a group holds the LDS
// offsets of its operands and the values of entries 4g..4g+3 (one stream for
// FP64 input, one with FP32-rounded values for FP32 input, and the latter
// with FP32 values for FP32 accumulation), a slot outside the chunk value 0
// and the chunk's first union row. The diagonal (entry 0) stays outside: the
// kernel takes it from the row itself. Built on the host from the
// operator's rows; needs fewer than 65536 strings.
static bool build_ss_blocks(int64_t N, int r, const std::vector<int32_t>& col, const std::vector<double>& val,
                            int R, std::vector<uint16_t>& uni, std::vector<uint16_t>& goff,
                            std::vector<int32_t>& binfo, std::vector<int32_t>& rbase, std::vector<SsGroup>& gs64,
                            std::vector<SsGroup>& gs32, std::vector<SsGroupF>& gsf, int* rc);
static int ensure_ss_blocks(casci_ctx* ctx, int spin)
{
    const bool b = spin == 1 && ctx->nb != ctx->na;
    casci_ctx::Blocks& bl = ctx->blk[b ? 1 : 0];
    if (bl.have) return CASCI_OK;
    const int64_t N = b ? ctx->Nb : ctx->Na;
    const int r = b ? ctx->rb : ctx->ra;
    // not available: the other widths serve
    if (!ctx->ops_sorted || N <= 0 || r <= 1 || N >= 65536) return CASCI_OK;
    const DBuf& dcol = b ? ctx->d_fb_col : ctx->d_fa_col;
    const DBuf& dval = b ? ctx->d_fb_val : ctx->d_fa_val;
    std::vector<int32_t> col((size_t)N * r);
    std::vector<double> val((size_t)N * r);
    HIPC(hipMemcpyAsync(col.data(), dcol.p, col.size() * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipMemcpyAsync(val.data(), dval.p, val.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    for (int64_t e0 = 0; e0 < N * (int64_t)r; e0 += r)
        for (int e = 1; e < r; ++e) {
            const int32_t J = col[(size_t)e0 + e];
            if (J < 0 || J >= N) return ctx->fail(CASCI_E_DEVICE, "same-spin operator: column out of range");
            if (e > 1 && J <= col[(size_t)e0 + e - 1])
                return ctx->fail(CASCI_E_DEVICE, "same-spin operator: row not in ascending column order");
        }
    std::vector<uint16_t> uni, goff;
    std::vector<int32_t> binfo, rbase;
    std::vector<SsGroup> gs64, gs32;
    std::vector<SsGroupF> gsf;
    // 32-row blocks stage fewer union rows per row; where a union of 32 rows
    // needs more than SS_BLK_MAXCH chunks, 16-row blocks; where those do too
    // (or a row has more groups than 16-bit offsets hold), no blocked form
    int R = 0;
    int64_t nblk = 0;
    for (int Rtry : {2 * SS_BLK_W, SS_BLK_W}) {
        int rc = CASCI_OK;
        if (build_ss_blocks(N, r, col, val, Rtry, uni, goff, binfo, rbase, gs64, gs32, gsf, &rc)) {
            R = Rtry;
            nblk = (N + R - 1) / R;
            break;
        }
        if (rc != CASCI_OK) return ctx->fail(rc, "same-spin operator too large for the row-blocked form");
    }
    if (R == 0) return CASCI_OK;  // the other widths serve
    HIPC(bl.uni.ensure(uni.size() * 2));
    HIPC(bl.binfo.ensure(binfo.size() * 4));
    HIPC(bl.goff.ensure(goff.size() * 2));
    HIPC(bl.rbase.ensure(rbase.size() * 4));
    HIPC(bl.gs64.ensure(gs64.size() * sizeof(SsGroup)));
    HIPC(bl.gs32.ensure(gs32.size() * sizeof(SsGroup)));
    HIPC(bl.gsf.ensure(gsf.size() * sizeof(SsGroupF)));
    HIPC(hipMemcpyAsync(bl.uni.p, uni.data(), uni.size() * 2, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipMemcpyAsync(bl.binfo.p, binfo.data(), binfo.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipMemcpyAsync(bl.goff.p, goff.data(), goff.size() * 2, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipMemcpyAsync(bl.rbase.p, rbase.data(), rbase.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipMemcpyAsync(bl.gs64.p, gs64.data(), gs64.size() * sizeof(SsGroup), hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipMemcpyAsync(bl.gs32.p, gs32.data(), gs32.size() * sizeof(SsGroup), hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipMemcpyAsync(bl.gsf.p, gsf.data(), gsf.size() * sizeof(SsGroupF), hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));  // pageable sources
    bl.nblk = nblk;
    bl.rows = R;
    bl.have = true;
    ++ctx->gen;  // captured graphs hold the operator without the blocks
    return CASCI_OK;
}

// The tables of the row-blocked form for blocks of R rows (the layout is
// described above ensure_ss_blocks). Returns false when a block's union needs
// more than SS_BLK_MAXCH chunks or a row more than 65535 groups (rc stays
// CASCI_OK), or when a table outgrows its 32-bit offsets (rc set).
static bool build_ss_blocks(int64_t N, int r, const std::vector<int32_t>& col, const std::vector<double>& val,
                            int R, std::vector<uint16_t>& uni, std::vector<uint16_t>& goff,
                            std::vector<int32_t>& binfo, std::vector<int32_t>& rbase, std::vector<SsGroup>& gs64,
                            std::vector<SsGroup>& gs32, std::vector<SsGroupF>& gsf, int* rc)
{
    const int CH = SS_BLK_CH;
    const int64_t nblk = (N + R - 1) / R;
    uni.clear();
    goff.clear();
    gs64.clear();
    gs32.clear();
    gsf.clear();
    binfo.assign((size_t)nblk * 4, 0);
    rbase.assign((size_t)N, 0);
    gs64.reserve((size_t)N * (r / 4 + 16));
    gs32.reserve((size_t)N * (r / 4 + 16));
    gsf.reserve((size_t)N * (r / 4 + 16));
    std::vector<int32_t> stamp((size_t)N, -1), where((size_t)N, 0);
    std::vector<int32_t> u;
    for (int64_t blk = 0; blk < nblk; ++blk) {
        const int64_t I0 = blk * R, I1 = std::min<int64_t>(N, I0 + R);
        u.clear();
        for (int64_t I = I0; I < I1; ++I)
            for (int e = 1; e < r; ++e) {
                const int32_t J = col[(size_t)I * r + e];
                if (stamp[J] != (int32_t)blk) {
                    stamp[J] = (int32_t)blk;
                    u.push_back(J);
                }
            }
        std::sort(u.begin(), u.end());
        for (size_t k = 0; k < u.size(); ++k) where[u[k]] = (int32_t)k;
        const int nU = (int)u.size();
        const int nch = (nU + CH - 1) / CH;
        if (nch > SS_BLK_MAXCH) return false;  // union too wide
        binfo[(size_t)blk * 4 + 0] = (int32_t)uni.size();
        binfo[(size_t)blk * 4 + 1] = nU;
        binfo[(size_t)blk * 4 + 2] = (int32_t)goff.size();
        binfo[(size_t)blk * 4 + 3] = nch;
        if (uni.size() + u.size() > 0x7fffffffu || goff.size() + (size_t)R * (nch + 1) > 0x7fffffffu) {
            *rc = CASCI_E_UNSUPPORTED;
            return false;
        }
        for (int32_t J : u) uni.push_back((uint16_t)J);
        for (int w = 0; w < R; ++w) {
            const int64_t I = I0 + w;
            if (I >= I1) {
                goff.insert(goff.end(), (size_t)nch + 1, 0);
                continue;
            }
            if (gs64.size() > 0x7fffffffu) {
                *rc = CASCI_E_UNSUPPORTED;
                return false;
            }
            rbase[(size_t)I] = (int32_t)gs64.size();
            const int32_t* cI = col.data() + (size_t)I * r;
            const double* vI = val.data() + (size_t)I * r;
            int e = 1;
            size_t ng = 0;
            for (int ch = 0; ch < nch; ++ch) {
                goff.push_back((uint16_t)ng);
                int ez = e;
                while (ez < r && where[cI[ez]] < (ch + 1) * CH) ++ez;
                for (int g = e & ~3; g < ez; g += 4) {
                    SsGroup a, b;
                    SsGroupF f;
                    for (int sl = 0; sl < 4; ++sl) {
                        const int x = g + sl;
                        const bool in = x >= e && x < ez;
                        const uint32_t q = (uint32_t)(in ? where[cI[x]] : ch * CH);
                        // row of the operand within the LDS chunk, times the row's bytes
                        a.off[sl] = b.off[sl] = f.off[sl] = (q % CH) * (uint32_t)SS_BLK_ROWB;
                        a.v[sl] = in ? vI[x] : 0.0;
                        f.v[sl] = in ? (float)vI[x] : 0.0f;
                        b.v[sl] = (double)f.v[sl];
                    }
                    gs64.push_back(a);
                    gs32.push_back(b);
                    gsf.push_back(f);
                    ++ng;
                }
                e = ez;
            }
            if (ng > 65535) return false;  // row too long for 16-bit group offsets
            goff.push_back((uint16_t)ng);
        }
    }
    if (uni.empty()) uni.push_back(0);
    if (gs64.empty()) {
        gs64.push_back(SsGroup{});
        gs32.push_back(SsGroup{});
        gsf.push_back(SsGroupF{});
    }
    return true;
}

// Autotuner of the same-spin gather: the strip width (lanes per gathered
// entry, 16/32/64) that is fastest for this string space, timed once per
// (device, norb, nalpha, nbeta, input precision) on the context's stream and
// cached for the process. The gather's summation order does not depend on
// the width, so the choice changes the speed only, never the result.
static std::mutex g_tune_mu;
static std::map<std::array<int, 5>, int> g_tune;

static int autotune_gather(casci_ctx* ctx, bool lowp, const double* C, const float* C32, int64_t ld32)
{
    // the choice depends on whether the row-blocked form is among the candidates
    const bool blk = ctx->blk[0].have;
    const std::array<int, 5> key = {ctx->device, ctx->norb, ctx->na, ctx->nb, (lowp ? 1 : 0) + (blk ? 2 : 0)};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            ctx->tune_lpe[lowp] = it->second;
            ctx->tune_blk[lowp] = blk;
            return CASCI_OK;
        }
    }
    hipStream_t st = ctx->stream;
    // timed on the first eighth of the rows (at least 2048): the same strips and
    // operator rows, a fraction of the cost on large spaces; the FP64 output of
    // those rows only (the FP32-storage build holds no full FP64 vector)
    const int64_t nt = std::min<int64_t>(ctx->Na, std::max<int64_t>(2048, ctx->Na / 8));
    HIPC(ctx->d_t1.ensure((size_t)nt * ctx->Nb * 8));
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return ctx->fail(CASCI_E_DEVICE, "hipEventCreate failed");
    }
    int best = 0;
    float best_ms = 0.f;
    hipError_t err = hipSuccess;
    static const int cand64[] = {SS_BLOCKED, 16, 32, 64, 128, 1602, 3202};
    static const int cand32[] = {SS_BLOCKED, 16, 32, 64, 128, 1602, 3202, 1604, 3204, 6404};
    // (the blocked width joins when its tables exist)
    const int* cand = (lowp ? cand32 : cand64) + (blk ? 0 : 1);
    const int ncand = (lowp ? 10 : 7) - (blk ? 0 : 1);
    for (int ci = 0; ci < ncand; ++ci) {
        const int lpe = cand[ci];
        auto run = [&]() {
            if (lowp)
                return launch_ss_gather_f32in(ss_op(ctx, 0), nt, ctx->Nb, C32, ld32, ctx->d_t1.as<double>(), 0.0,
                                              0, st, lpe);
            return launch_ss_gather_f64(ss_op(ctx, 0), nt, ctx->Nb, C, ctx->d_t1.as<double>(), 0.0, 0, st, lpe);
        };
        if ((err = run()) != hipSuccess) break;  // warm-up
        if ((err = hipEventRecord(e0, st)) != hipSuccess) break;
        for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) err = run();
        if (err != hipSuccess || (err = hipEventRecord(e1, st)) != hipSuccess) break;
        if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.f;
        if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        if (best == 0 || ms < best_ms) {
            best = lpe;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPC(err);
    ctx->tune_lpe[lowp] = best;
    ctx->tune_blk[lowp] = blk;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    return CASCI_OK;
}

// Autotuner of the FP64 alpha-beta layout (M tiles per wave, sigma-row chunks
// in LDS): the candidates with a kernel variant for this shape are timed on
// the first eighth of the alpha strings (at least 256) of the build that
// needs it, once per (device, norb, nalpha, nbeta, pair set) and cached for
// the process. The fixed-point sums make every layout give the same bits.
static std::map<std::array<int, 5>, int> g_tune_ab;

static int autotune_ab_f64(casci_ctx* ctx, int full, const AbParams& p, const double* Vt, const double* C,
                           const double* rowmax, double* out)
{
    const std::array<int, 5> key = {ctx->device, ctx->norb, ctx->na, ctx->nb, full};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_ab.find(key);
        if (it != g_tune_ab.end()) {
            ctx->tune_ab[full] = it->second;
            return CASCI_OK;
        }
    }
    hipStream_t st = ctx->stream;
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return ctx->fail(CASCI_E_DEVICE, "hipEventCreate failed");
    }
    AbParams q = p;
    q.Na = std::min<int64_t>(p.Na, std::max<int64_t>(256, p.Na / 8));
    int best = 0;
    float best_ms = 0.f;
    hipError_t err = hipSuccess;
    static const int cand[] = {11, 21, 12, 22};
    for (int code : cand) {
        // a layout without a kernel variant for this shape is refused before
        // any launch: skipped
        if (launch_ab_f64(q, Vt, C, rowmax, out, st, code) != hipSuccess) {
            set_launch_reason("");
            continue;
        }
        if ((err = hipEventRecord(e0, st)) != hipSuccess) break;
        for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) err = launch_ab_f64(q, Vt, C, rowmax, out, st, code);
        if (err != hipSuccess || (err = hipEventRecord(e1, st)) != hipSuccess) break;
        if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.f;
        if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        if (best == 0 || ms < best_ms) {
            best = code;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPC(err);
    if (best == 0) return ctx->fail(CASCI_E_UNSUPPORTED, "alpha-beta: no FP64 layout runs this shape");
    ctx->tune_ab[full] = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_ab[key] = best;
    return CASCI_OK;
}

// Vector-sized work buffers of one sigma build. sigma_dev fills them from the
// context's own (growing) buffers, or takes them from the caller: the
// allocation-free entry point passes slices of the library's static scratch.
struct SigmaWork {
    double* t1 = nullptr;      // C^T (general vectors, nbeta > 0): Nd
    double* t2 = nullptr;      // beta-beta gather on C^T: Nd
    double* t3 = nullptr;      // alpha-beta term: Nd
    double* rowmax = nullptr;  // FP64 alpha-beta: max |C(J, :)| per alpha string: Na
    float* c32 = nullptr;      // FP32 copy of C (low-precision builds): Na x lowp_ld(1, Nb)
    void* clp = nullptr;       // BF16 copy of C (BF16 builds): Na x lowp_ld(2, Nb)
};

// bytes of the work buffers one build needs (each piece 256-byte aligned), and
// their placement in one block of memory
static size_t sigma_work_layout(const casci_ctx* ctx, int ab_prec, int parity, unsigned char* base, SigmaWork* w)
{
    const int64_t Na = ctx->Na, Nb = ctx->Nb, Nd = ctx->Nd;
    const bool lowp = ab_prec != CASCI_F64;
    const bool has_ab = ctx->na > 0 && ctx->nb > 0;
    size_t off = 0;
    auto take = [&](size_t bytes) -> unsigned char* {
        unsigned char* p = base ? base + off : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    SigmaWork x;
    if (parity == 0 && ctx->nb > 0) {
        x.t1 = (double*)take((size_t)Nd * 8);
        x.t2 = (double*)take((size_t)Nd * 8);
    }
    if (has_ab) x.t3 = (double*)take((size_t)Nd * 8);
    if (has_ab) x.rowmax = (double*)take((size_t)Na * 8);
    if (lowp) x.c32 = (float*)take((size_t)Na * lowp_ld(1, Nb) * 4);
    if (lowp && has_ab && ab_prec == CASCI_BF16) x.clp = take((size_t)Na * lowp_ld(2, Nb) * 2);
    if (w) *w = x;
    return off;
}

// sigma = (H + lambda S^2) C on device vectors (FP64 storage).
// parity = +1 / -1 declares C = +-C^T (nalpha = nbeta only): transposition
// commutes with H, so sigma_bb = parity * sigma_aa^T and one same-spin gather
// serves both spins. parity = 0: general C. ab_prec != F64 also reads the
// same-spin gather operand from an FP32 copy of C; the accumulation stays
// FP64, except in the row-blocked gather of a BF16 build, which sums in FP32
// (relative error ~1e-6 against the ~1e-3 of the BF16 alpha-beta part).
// The alpha-beta contraction writes its own buffer, added in by the final pass
// (with parity fused into the S + p S^T symmetrisation). Running it on a
// second stream beside the gathers was measured not to help: each slows the
// other by as much as the overlap gains.
// work = nullptr: the context's buffers (allocated or grown as needed, the
// tables built, the gather autotuned). work given: nothing is allocated; the
// tables must exist and the gather uses its tuned (or default) strip width.
static int sigma_dev(casci_ctx* ctx, const double* C, double* S, int ab_prec, double lambda,
                     int parity = 0, const SigmaWork* work = nullptr)
{
    hipStream_t st = ctx->stream;
    const int64_t Na = ctx->Na, Nb = ctx->Nb, Nd = ctx->Nd;
    const double ms = 0.5 * (ctx->na - ctx->nb);
    const double shift = ctx->ecore + lambda * (ms * ms + ms + ctx->nb);
    const bool prof = ctx->profiling;
    const bool lowp = ab_prec != CASCI_F64;
    const bool has_ab = ctx->na > 0 && ctx->nb > 0;
    const bool alloc = work == nullptr;
    if (parity != 0 && ctx->na != ctx->nb) return ctx->fail(CASCI_E_ARG, "parity needs nalpha == nbeta");
    set_launch_reason("");
    SigmaWork w;
    if (alloc) {
        if (parity == 0 && ctx->nb > 0) {
            HIPC(ctx->d_t1.ensure((size_t)Nd * 8));
            HIPC(ctx->d_t2.ensure((size_t)Nd * 8));
            w.t1 = ctx->d_t1.as<double>();
            w.t2 = ctx->d_t2.as<double>();
        }
        if (has_ab) {
            HIPC(ctx->d_t3.ensure((size_t)Nd * 8));
            w.t3 = ctx->d_t3.as<double>();
        }
        if (has_ab) {
            HIPC(ctx->d_rowmax.ensure((size_t)Na * 8));
            w.rowmax = ctx->d_rowmax.as<double>();
        }
        if (lowp) {
            HIPC(ctx->d_c32.ensure((size_t)Na * lowp_ld(1, Nb) * 4));
            w.c32 = ctx->d_c32.as<float>();
        }
        if (lowp && has_ab && ab_prec == CASCI_BF16) {
            HIPC(ctx->d_clp.ensure((size_t)Na * lowp_ld(2, Nb) * 2));
            w.clp = ctx->d_clp.p;
        }
    } else {
        w = *work;
    }
    auto mark = [&](int i, hipStream_t s) -> int {
        if (prof) HIPC(hipEventRecord(ctx->pev[i], s));
        return CASCI_OK;
    };
    CHECK_RC(mark(0, st));
    // inputs in the arithmetic's types (stream order: before the fork)
    const int64_t ld32 = lowp_ld(1, Nb), ld16 = lowp_ld(2, Nb);
    if (lowp) {
        HIPC(launch_convert_lowp(1, C, w.c32, Na, Nb, ld32, st));
        if (has_ab && ab_prec == CASCI_BF16) HIPC(launch_convert_lowp(2, C, w.clp, Na, Nb, ld16, st));
    }
    // alpha-beta, overwriting t3
    if (has_ab) {
        CHECK_RC(mark(3, st));
        const bool full = lambda != 0.0 || !ctx->eri8;
        CHECK_RC(ensure_targets(ctx, full, alloc));
        AbParams p = ab_params(ctx, full);
        p.overwrite = 1;
        if (!lowp) {
            const DBuf& vt = full ? ctx->d_vt_full : ctx->d_vt_sym;
            HIPC(launch_row_absmax(C, Na, Nb, w.rowmax, st));
            if (alloc && ctx->tune_ab[full] == 0)
                CHECK_RC(autotune_ab_f64(ctx, full, p, vt.as<double>(), C, w.rowmax, w.t3));
            HIPC(launch_ab_f64(p, vt.as<double>(), C, w.rowmax, w.t3, st, ctx->tune_ab[full]));
        } else {
            const DBuf* lp = full ? ctx->d_vt_full_lp : ctx->d_vt_sym_lp;
            if (ab_prec == CASCI_BF16 && !full && ab_bf16_fixed_fits(Nb, ctx->sa, p.Mp)) {
                // scatter from the accumulators into a fixed-point row (no reduction table)
                CHECK_RC(ensure_tg16(ctx, alloc));
                HIPC(launch_row_absmax(C, Na, Nb, w.rowmax, st));
                HIPC(launch_ab_bf16_fixed(p, lp[1].p, w.clp, ld16, w.rowmax, ctx->d_tg16.as<uint16_t>(), w.t3, st));
            } else {
                AbReduce red;
                CHECK_RC(ensure_reduce(ctx, full, &red, alloc));
                if (ab_prec == CASCI_F32)
                    HIPC(launch_ab_lowp(p, red, 1, lp[0].p, w.c32, ld32, w.t3, st));
                else
                    HIPC(launch_ab_lowp(p, red, 2, lp[1].p, w.clp, ld16, w.t3, st));
            }
        }
        CHECK_RC(mark(4, st));
    }
    const double s_aa = parity != 0 ? 0.5 * shift : shift;  // halved: S + p S^T doubles it
    // the strip width changes only the speed, not the sums (fixed summation order)
    if (alloc) CHECK_RC(ensure_ss_blocks(ctx, 0));
    // tuned once, and again once the row-blocked form exists if an earlier
    // build (the FP32-storage one) tuned without it
    if (alloc && (ctx->tune_lpe[lowp ? 1 : 0] == 0 || (ctx->blk[0].have && !ctx->tune_blk[lowp ? 1 : 0])))
        CHECK_RC(autotune_gather(ctx, lowp, C, w.c32, ld32));
    const int lpe = ctx->tune_lpe[lowp ? 1 : 0];
    if (lowp)
        HIPC(launch_ss_gather_f32in(ss_op(ctx, 0), Na, Nb, w.c32, ld32, S, s_aa, 0, st, lpe, ab_prec == CASCI_BF16));
    else
        HIPC(launch_ss_gather_f64(ss_op(ctx, 0), Na, Nb, C, S, s_aa, 0, st, lpe));
    CHECK_RC(mark(1, st));
    if (parity == 0 && ctx->nb > 0) {
        const bool same = ctx->nb == ctx->na;
        HIPC(launch_transpose_f64(C, w.t1, Na, Nb, 0, 1.0, st));
        HIPC(launch_ss_gather_f64(ss_op(ctx, 1), Nb, Na, w.t1, w.t2, 0.0, 0, st, same && !lowp ? lpe : 0));
        HIPC(launch_transpose_f64(w.t2, S, Nb, Na, 1, 1.0, st));
    }
    CHECK_RC(mark(2, st));
    if (parity != 0)
        HIPC(launch_sym_add(S, Na, parity, 1.0, st, has_ab ? w.t3 : nullptr));
    else if (has_ab)
        HIPC(launch_axpby_f64(1.0, w.t3, 1.0, S, Nd, st));
    CHECK_RC(mark(5, st));
    if (prof) {
        HIPC(hipEventSynchronize(ctx->pev[5]));
        float t_aa = 0, t_bb = 0, t_ab = 0, t_tot = 0, t_end = 0, t_cv = 0;
        HIPC(hipEventElapsedTime(&t_cv, ctx->pev[0], ctx->pev[3]));  // conversions of C
        HIPC(hipEventElapsedTime(&t_aa, ctx->pev[4], ctx->pev[1]));
        t_aa += t_cv;
        HIPC(hipEventElapsedTime(&t_bb, ctx->pev[1], ctx->pev[2]));
        if (has_ab) HIPC(hipEventElapsedTime(&t_ab, ctx->pev[3], ctx->pev[4]));
        HIPC(hipEventElapsedTime(&t_end, ctx->pev[2], ctx->pev[5]));
        HIPC(hipEventElapsedTime(&t_tot, ctx->pev[0], ctx->pev[5]));
        // [0..5]: FP64 builds, [6..11]: low-precision builds; each: alpha-alpha
        // gather (with the conversions of C), beta-beta work, alpha-beta
        // contraction, final combination, whole build, number of builds
        double* pr = ctx->prof + (lowp ? 6 : 0);
        pr[0] += t_aa;
        pr[1] += t_bb;
        pr[2] += t_ab;
        pr[3] += t_end;
        pr[4] += t_tot;
        if (lowp) ctx->prof[12] += t_cv;  // the conversions alone (already in pr[0])
        pr[5] += 1;
    }
    return CASCI_OK;
}

// sigma = H C for an FP32-stored vector, without FP64 copies of the vector
// (the footprint that lets CAS(18e,18o) vectors, 9.5 GB each in FP32, be
// processed with room to spare). C32, S32: device, Na x Nb FP32. The
// same-spin gathers accumulate in FP64 registers and store FP32; the
// alpha-beta term (FP32 or BF16 MFMA, FP32 accumulation) is added into S32.
// Timed parts go to the low-precision profile slots.
// Width of the FP32-storage build's gather (FP32 in and out), timed on the
// whole space with the build's own kernel writing into S32 (overwritten by
// the build afterwards): on the first eighth of the rows the FP64-output
// launches the other tuner times ranked the widths differently at
// CAS(18,18) (64 lanes there, 1.88 s in full, against 1.07 s for 3204).
// Cached per (device, norb, nalpha, nbeta) for the process.
static int autotune_gather_f32s(casci_ctx* ctx, const float* C32, float* S32)
{
    const bool blk = ctx->blk[0].have;
    const std::array<int, 5> key = {ctx->device, ctx->norb, ctx->na, ctx->nb, 4 + (blk ? 2 : 0)};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            ctx->tune_lpe[1] = it->second;
            ctx->tune_blk[1] = blk;
            return CASCI_OK;
        }
    }
    hipStream_t st = ctx->stream;
    hipEvent_t e0, e1;
    HIPC(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return ctx->fail(CASCI_E_DEVICE, "hipEventCreate failed");
    }
    static const int cand[] = {SS_BLOCKED, 64, 128, 1604, 3204, 6404};
    int best = 0;
    float best_ms = 0.f;
    hipError_t err = hipSuccess;
    for (int ci = blk ? 0 : 1; ci < 6; ++ci) {
        const int lpe = cand[ci];
        if ((err = hipEventRecord(e0, st)) != hipSuccess) break;
        err = launch_ss_gather_f32(ss_op(ctx, 0), ctx->Na, ctx->Nb, C32, S32, 0.0, 0, st, lpe);
        if (err != hipSuccess || (err = hipEventRecord(e1, st)) != hipSuccess) break;
        if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.f;
        if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        if (best == 0 || ms < best_ms) {
            best = lpe;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    HIPC(err);
    ctx->tune_lpe[1] = best;
    ctx->tune_blk[1] = blk;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
    return CASCI_OK;
}

static int sigma_dev_f32(casci_ctx* ctx, const float* C32, float* S32, int ab_prec)
{
    hipStream_t st = ctx->stream;
    const int64_t Na = ctx->Na, Nb = ctx->Nb, Nd = ctx->Nd;
    const double ms = 0.5 * (ctx->na - ctx->nb);
    (void)ms;
    const double shift = ctx->ecore;
    const bool prof = ctx->profiling;
    const bool has_ab = ctx->na > 0 && ctx->nb > 0;
    set_launch_reason("");
    auto mark = [&](int i) -> int {
        if (prof) HIPC(hipEventRecord(ctx->pev[i], st));
        return CASCI_OK;
    };
    CHECK_RC(mark(0));
    CHECK_RC(mark(3));
    // the FP32-input width, tuned on this build's own kernel if no build has
    // tuned it yet
    if (ctx->tune_lpe[1] == 0) CHECK_RC(autotune_gather_f32s(ctx, C32, S32));
    const int lpe = ctx->tune_lpe[1];
    // alpha-alpha: S32 = F_a C + shift C
    HIPC(launch_ss_gather_f32(ss_op(ctx, 0), Na, Nb, C32, S32, shift, 0, st, lpe));
    CHECK_RC(mark(4));
    CHECK_RC(mark(1));
    // beta-beta: S32 += (F_b C^T)^T through two FP32 transposes
    if (ctx->nb > 0) {
        HIPC(ctx->d_t1.ensure((size_t)Nd * 4));
        HIPC(ctx->d_t2.ensure((size_t)Nd * 4));
        const bool same = ctx->nb == ctx->na;
        HIPC(launch_transpose_f32(C32, ctx->d_t1.as<float>(), Na, Nb, 0, st));
        HIPC(launch_ss_gather_f32(ss_op(ctx, 1), Nb, Na, ctx->d_t1.as<float>(), ctx->d_t2.as<float>(), 0.0, 0, st,
                                  same ? lpe : 0));
        HIPC(launch_transpose_f32(ctx->d_t2.as<float>(), S32, Nb, Na, 1, st));
    }
    CHECK_RC(mark(2));
    // alpha-beta, added into S32
    if (has_ab) {
        const bool full = !ctx->eri8;
        AbParams p = ab_params(ctx, full);
        p.overwrite = 0;
        AbReduce red;
        CHECK_RC(ensure_targets(ctx, full));
        CHECK_RC(ensure_reduce(ctx, full, &red));
        const int pr = ab_prec == CASCI_F32 ? 1 : 2;
        const int64_t ld = lowp_ld(pr, Nb);
        const void* Cs = C32;
        if (pr == 2 || ld != Nb) {
            DBuf& buf = pr == 1 ? ctx->d_c32 : ctx->d_clp;
            HIPC(buf.ensure((size_t)Na * ld * (pr == 1 ? 4 : 2)));
            HIPC(launch_convert_lowp_f32in(pr, C32, buf.p, Na, Nb, ld, st));
            Cs = buf.p;
        }
        HIPC(launch_ab_lowp(p, red, pr, (full ? ctx->d_vt_full_lp : ctx->d_vt_sym_lp)[pr - 1].p, Cs, ld, S32, st));
    }
    CHECK_RC(mark(5));
    if (prof) {
        HIPC(hipEventSynchronize(ctx->pev[5]));
        float t_aa = 0, t_bb = 0, t_ab = 0, t_tot = 0;
        HIPC(hipEventElapsedTime(&t_aa, ctx->pev[0], ctx->pev[1]));
        HIPC(hipEventElapsedTime(&t_bb, ctx->pev[1], ctx->pev[2]));
        HIPC(hipEventElapsedTime(&t_ab, ctx->pev[2], ctx->pev[5]));
        HIPC(hipEventElapsedTime(&t_tot, ctx->pev[0], ctx->pev[5]));
        double* q = ctx->prof + 6;
        q[0] += t_aa;
        q[1] += t_bb;
        q[2] += t_ab;
        q[4] += t_tot;
        q[5] += 1;
    }
    return CASCI_OK;
}

// Device buffers a captured sigma build reads or writes; a graph is replayed
// only while all of them are where they were at capture.
static std::vector<void*> sigma_buffers(const casci_ctx* ctx)
{
    std::vector<void*> v = {ctx->d_t1.p, ctx->d_t2.p, ctx->d_t3.p, ctx->d_c32.p, ctx->d_clp.p, ctx->d_fa_col.p,
            ctx->d_fa_val.p, ctx->d_fb_col.p, ctx->d_fb_val.p, ctx->d_vt_sym.p, ctx->d_vt_full.p,
            ctx->d_vt_sym_lp[0].p, ctx->d_vt_sym_lp[1].p, ctx->d_vt_full_lp[0].p, ctx->d_vt_full_lp[1].p,
            ctx->d_tg_sym.p, ctx->d_tg_full.p, ctx->red_sym.tab.p, ctx->red_sym.tinfo.p, ctx->red_full.tab.p,
            ctx->red_full.tinfo.p, ctx->d_la_j.p, ctx->d_la_pq.p, ctx->d_lb_j.p, ctx->d_bstr.p,
            ctx->d_pairs_sym.p, ctx->d_pairs_full.p, ctx->d_gin.p, ctx->d_gout.p, ctx->d_fa_c16.p,
            ctx->d_fa_v32.p, ctx->d_fb_c16.p, ctx->d_fb_v32.p, ctx->d_rowmax.p, ctx->d_tg16.p};
    for (const auto& bl : ctx->blk)
        for (const DBuf* d : {&bl.uni, &bl.binfo, &bl.goff, &bl.rbase, &bl.gs64, &bl.gs32, &bl.gsf}) v.push_back(d->p);
    return v;
}

// sigma_dev replayed from a captured HIP graph: one launch per build instead
// of one per kernel (what dominates for small active spaces). C is staged
// into d_gin and the result copied out of d_gout around the replay. The
// first build of a (precision, parity, lambda) runs eagerly once (it
// allocates, builds the tables and autotunes), then the same build is
// captured. The captured graph holds no memset nodes.
static int sigma_graph(casci_ctx* ctx, const double* C, double* S, int ab_prec, double lambda, int parity)
{
    hipStream_t st = ctx->stream;
    const size_t vb = (size_t)ctx->Nd * 8;
    HIPC(ctx->d_gin.ensure(vb));
    HIPC(ctx->d_gout.ensure(vb));
    // drop stale graphs
    const std::vector<void*> now = sigma_buffers(ctx);
    for (size_t i = 0; i < ctx->graphs.size();) {
        auto& g = ctx->graphs[i];
        if (g.gen != ctx->gen || g.sig != now) {
            (void)hipGraphExecDestroy(g.exec);
            ctx->graphs.erase(ctx->graphs.begin() + i);
        } else {
            ++i;
        }
    }
    hipGraphExec_t exec = nullptr;
    for (auto& g : ctx->graphs)
        if (g.prec == ab_prec && g.parity == parity && g.lambda == lambda) exec = g.exec;
    HIPC(hipMemcpyAsync(ctx->d_gin.p, C, vb, hipMemcpyDeviceToDevice, st));
    if (!exec) {
        CHECK_RC(sigma_dev(ctx, ctx->d_gin.as<double>(), ctx->d_gout.as<double>(), ab_prec, lambda, parity));
        HIPC(hipStreamSynchronize(st));
        const bool prof = ctx->profiling;
        ctx->profiling = false;
        HIPC(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const int rc = sigma_dev(ctx, ctx->d_gin.as<double>(), ctx->d_gout.as<double>(), ab_prec, lambda, parity);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(st, &graph);
        ctx->profiling = prof;
        if (rc < 0) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        HIPC(ec);
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPC(ei);
        casci_ctx::Graph g;
        g.prec = ab_prec;
        g.parity = parity;
        g.lambda = lambda;
        g.gen = ctx->gen;
        g.sig = sigma_buffers(ctx);
        g.exec = exec;
        ctx->graphs.push_back(g);
    }
    HIPC(hipGraphLaunch(exec, st));
    HIPC(hipMemcpyAsync(S, ctx->d_gout.p, vb, hipMemcpyDeviceToDevice, st));
    return CASCI_OK;
}

extern "C" int casci_set_tuning(casci_ctx* ctx, int f64_lpe, int f32in_lpe)
{
    if (!ctx) return CASCI_E_ARG;
    for (int v : {f64_lpe, f32in_lpe})
        if (v != 0 && v != 16 && v != 32 && v != 64 && v != 128 && v != 1602 && v != 3202 && v != 1604 &&
            v != 3204 && v != 6404 && v != SS_BLOCKED)
            return ctx->fail(CASCI_E_ARG,
                             "strip width code must be 0, 16, 32, 64, 128, 1602, 3202, 1604, 3204, 6404 or 99");
    ctx->tune_lpe[0] = f64_lpe;
    ctx->tune_lpe[1] = f32in_lpe;
    ctx->tune_blk[0] = ctx->tune_blk[1] = true;  // a width set by the caller is kept
    ++ctx->gen;  // captured graphs hold the old choice
    return CASCI_OK;
}

extern "C" int casci_get_tuning(casci_ctx* ctx, int* out)
{
    if (!ctx || !out) return CASCI_E_ARG;
    out[0] = ctx->tune_lpe[0];
    out[1] = ctx->tune_lpe[1];
    return CASCI_OK;
}

extern "C" int casci_set_ab_layout(casci_ctx* ctx, int pairs, int code)
{
    if (!ctx) return CASCI_E_ARG;
    if (pairs != 0 && pairs != 1) return ctx->fail(CASCI_E_ARG, "pairs must be 0 (r <= s) or 1 (all ordered pairs)");
    const int mt = code / 10, split = code % 10;
    if (code != 0 && (code < 0 || mt < 1 || mt > 2 || split < 1 || split > 4))
        return ctx->fail(CASCI_E_ARG, "FP64 alpha-beta layout code must be 0 or 10 MT + split (MT 1..2, split 1..4)");
    ctx->tune_ab[pairs] = code;
    ++ctx->gen;  // captured graphs hold the old choice
    return CASCI_OK;
}

extern "C" int casci_get_ab_layout(casci_ctx* ctx, int* out)
{
    if (!ctx || !out) return CASCI_E_ARG;
    out[0] = ctx->tune_ab[0];
    out[1] = ctx->tune_ab[1];
    return CASCI_OK;
}

// sizes and offsets of the option / info structs (for bindings to check their layout)
extern "C" int casci_abi_layout(int64_t* out, int n)
{
    if (!out || n < 6) return CASCI_E_ARG;
    out[0] = (int64_t)sizeof(casci_davidson_opts);
    out[1] = (int64_t)sizeof(casci_davidson_info);
    out[2] = (int64_t)offsetof(casci_davidson_opts, progress);
    out[3] = (int64_t)offsetof(casci_davidson_info, residual);
    out[4] = (int64_t)offsetof(casci_davidson_info, hist_energy);
    out[5] = (int64_t)offsetof(casci_davidson_info, hist_len);
    return CASCI_OK;
}

extern "C" int casci_profile_enable(casci_ctx* ctx, int on)
{
    if (!ctx) return CASCI_E_ARG;
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    if (on) {
        for (hipEvent_t& e : ctx->pev)
            if (!e) HIPC(hipEventCreate(&e));
        for (double& x : ctx->prof) x = 0.0;
    }
    ctx->profiling = on != 0;
    return CASCI_OK;
}

extern "C" int casci_profile_read(const casci_ctx* ctx, double* out)
{
    if (!ctx || !out) return CASCI_E_ARG;
    for (int i = 0; i < 16; ++i) out[i] = ctx->prof[i];
    return CASCI_OK;
}

extern "C" int casci_get_same_spin_operator(casci_ctx* ctx, int spin, int32_t* col, double* val)
{
    if (!ctx) return CASCI_E_ARG;
    if (spin != 0 && spin != 1) return ctx->fail(CASCI_E_ARG, "spin must be 0 or 1");
    if (!col || !val) return ctx->fail(CASCI_E_ARG, "col and val must not be NULL");
    DeviceGuard g(ctx->device);
    CHECK_RC(ensure_prepared(ctx, 0.0));
    const bool same = ctx->nb == ctx->na;
    const int64_t N = spin ? ctx->Nb : ctx->Na;
    const int r = spin ? ctx->rb : ctx->ra;
    const DBuf& dc = (spin && !same) ? ctx->d_fb_col : ctx->d_fa_col;
    const DBuf& dv = (spin && !same) ? ctx->d_fb_val : ctx->d_fa_val;
    const size_t cnt = (size_t)N * r;
    std::vector<int32_t> c(cnt);
    std::vector<double> v(cnt);
    HIPC(hipMemcpyAsync(c.data(), dc.p, cnt * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipMemcpyAsync(v.data(), dv.p, cnt * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    std::vector<int> idx(r);
    for (int64_t I = 0; I < N; ++I) {
        for (int k = 0; k < r; ++k) idx[k] = k;
        const int32_t* cr = c.data() + I * r;
        std::sort(idx.begin(), idx.end(), [&](int a, int b) { return cr[a] < cr[b]; });
        for (int k = 0; k < r; ++k) {
            col[I * r + k] = cr[idx[k]];
            val[I * r + k] = v[I * r + idx[k]];
        }
    }
    return CASCI_OK;
}

extern "C" int casci_get_diagonal(casci_ctx* ctx, double* out, int mem)
{
    if (!ctx) return CASCI_E_ARG;
    if (!out) return ctx->fail(CASCI_E_ARG, "out is NULL");
    if (mem != CASCI_MEM_HOST && mem != CASCI_MEM_DEVICE) return ctx->fail(CASCI_E_ARG, "bad mem flag");
    DeviceGuard g(ctx->device);
    CHECK_RC(ensure_prepared(ctx, 0.0));
    HIPC(hipMemcpyAsync(out, ctx->d_diag.p, (size_t)ctx->Nd * 8,
                        mem == CASCI_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                        ctx->stream));
    if (mem == CASCI_MEM_HOST) HIPC(hipStreamSynchronize(ctx->stream));
    return CASCI_OK;
}

static int lowest_diag(casci_ctx* ctx, int64_t want, std::vector<int64_t>& out);

extern "C" int casci_lowest_diagonal(casci_ctx* ctx, int64_t want, int64_t* out)
{
    if (!ctx) return CASCI_E_ARG;
    if (!out || want < 0) return ctx->fail(CASCI_E_ARG, "out is NULL or want < 0");
    if (ctx->validate_only) return ctx->fail(CASCI_E_UNSUPPORTED, kValidateOnly);
    if (!ctx->has_strings) return ctx->fail(CASCI_E_ARG, "build strings first");
    if (want > ctx->Nd) return ctx->fail(CASCI_E_ARG, "want exceeds the number of determinants");
    DeviceGuard g(ctx->device);
    CHECK_RC(ensure_prepared(ctx, 0.0));
    std::vector<int64_t> v;
    CHECK_RC(lowest_diag(ctx, want, v));
    std::copy(v.begin(), v.end(), out);
    return CASCI_OK;
}

static int check_vec_args(casci_ctx* ctx, const void* C, const void* S, int dtype, int ab_prec, int mem)
{
    if (!C || !S) return ctx->fail(CASCI_E_ARG, "C and sigma must not be NULL");
    if (C == S) return ctx->fail(CASCI_E_ARG, "C and sigma must not overlap");
    if (dtype != CASCI_F64 && dtype != CASCI_F32) return ctx->fail(CASCI_E_ARG, "dtype must be F64 or F32");
    if (ab_prec != CASCI_F64 && ab_prec != CASCI_F32 && ab_prec != CASCI_BF16)
        return ctx->fail(CASCI_E_ARG, "ab_prec must be F64, F32 or BF16");
    if (mem != CASCI_MEM_HOST && mem != CASCI_MEM_DEVICE) return ctx->fail(CASCI_E_ARG, "bad mem flag");
    return CASCI_OK;
}

// sigma of a host or device vector (FP64 or FP32 storage); parity != 0
// declares C = parity C^T (nalpha = nbeta) and takes the one-gather path
static int sigma_impl(casci_ctx* ctx, const void* C, void* sigma, int dtype, int ab_prec, int parity, int mem)
{
    if (!ctx) return CASCI_E_ARG;
    CHECK_RC(check_vec_args(ctx, C, sigma, dtype, ab_prec, mem));
    if (!ctx->has_ints) return ctx->fail(CASCI_E_STATE, "set_integrals first");
    if (!ctx->has_strings) return ctx->fail(CASCI_E_STATE, "build_strings first");
    if (parity != 0 && parity != 1 && parity != -1) return ctx->fail(CASCI_E_ARG, "parity must be +1 or -1");
    if (parity != 0 && ctx->na != ctx->nb) return ctx->fail(CASCI_E_ARG, "parity needs nalpha == nbeta");
    if (parity != 0 && dtype != CASCI_F64) return ctx->fail(CASCI_E_ARG, "parity needs FP64 storage");
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    CHECK_RC(ensure_prepared(ctx, 0.0));
    const size_t Nd = (size_t)ctx->Nd;
    const size_t esz = dtype == CASCI_F64 ? 8 : 4;
    hipStream_t st = ctx->stream;
    if (dtype == CASCI_F32 && mem == CASCI_MEM_DEVICE && ab_prec != CASCI_F64)
        return sigma_dev_f32(ctx, (const float*)C, (float*)sigma, ab_prec);
    const double* cin;
    double* sout;
    if (dtype == CASCI_F64 && mem == CASCI_MEM_DEVICE) {
        cin = (const double*)C;
        sout = (double*)sigma;
    } else {
        HIPC(ctx->d_vin.ensure(Nd * 8));
        HIPC(ctx->d_vout.ensure(Nd * 8));
        cin = ctx->d_vin.as<double>();
        sout = ctx->d_vout.as<double>();
        if (dtype == CASCI_F64) {
            HIPC(hipMemcpyAsync(ctx->d_vin.p, C, Nd * 8, hipMemcpyHostToDevice, st));
        } else {
            const float* src = (const float*)C;
            if (mem == CASCI_MEM_HOST) {
                HIPC(ctx->d_vout.ensure(Nd * 8));
                HIPC(hipMemcpyAsync(ctx->d_vout.p, C, Nd * esz, hipMemcpyHostToDevice, st));
                src = ctx->d_vout.as<float>();
            }
            HIPC(launch_convert_f32_to_f64(src, ctx->d_vin.as<double>(), (int64_t)Nd, st));
        }
    }
    CHECK_RC(sigma_dev(ctx, cin, sout, ab_prec, 0.0, parity));
    if (!(dtype == CASCI_F64 && mem == CASCI_MEM_DEVICE)) {
        if (dtype == CASCI_F64) {
            HIPC(hipMemcpyAsync(sigma, sout, Nd * 8, hipMemcpyDeviceToHost, st));
        } else if (mem == CASCI_MEM_DEVICE) {
            HIPC(launch_convert_f64_to_f32(sout, (float*)sigma, (int64_t)Nd, st));
        } else {
            HIPC(launch_convert_f64_to_f32(sout, (float*)ctx->d_vin.p, (int64_t)Nd, st));
            HIPC(hipMemcpyAsync(sigma, ctx->d_vin.p, Nd * 4, hipMemcpyDeviceToHost, st));
        }
        if (mem == CASCI_MEM_HOST) HIPC(hipStreamSynchronize(st));
    }
    return CASCI_OK;
}

extern "C" int casci_sigma(casci_ctx* ctx, const void* C, void* sigma, int dtype, int ab_prec, int mem)
{
    return sigma_impl(ctx, C, sigma, dtype, ab_prec, 0, mem);
}

extern "C" int casci_sigma_parity(casci_ctx* ctx, const double* C, double* sigma, int ab_prec, int parity, int mem)
{
    if (!ctx) return CASCI_E_ARG;
    if (parity == 0) return ctx->fail(CASCI_E_ARG, "parity must be +1 or -1");
    return sigma_impl(ctx, C, sigma, CASCI_F64, ab_prec, parity, mem);
}

extern "C" int casci_sigma_noalloc(casci_ctx* ctx, const double* C, double* sigma, int ab_prec, int parity)
{
    if (!ctx) return CASCI_E_ARG;
    if (!C || !sigma) return ctx->fail(CASCI_E_ARG, "C and sigma must not be NULL");
    if (C == sigma) return ctx->fail(CASCI_E_ARG, "C and sigma must not overlap");
    if (ab_prec != CASCI_F64 && ab_prec != CASCI_F32 && ab_prec != CASCI_BF16)
        return ctx->fail(CASCI_E_ARG, "ab_prec must be F64, F32 or BF16");
    if (parity != 0 && parity != 1 && parity != -1) return ctx->fail(CASCI_E_ARG, "parity must be 0, +1 or -1");
    if (!ctx->has_ints) return ctx->fail(CASCI_E_STATE, "set_integrals first");
    if (!ctx->has_strings) return ctx->fail(CASCI_E_STATE, "build_strings first");
    if (parity != 0 && ctx->na != ctx->nb) return ctx->fail(CASCI_E_ARG, "parity needs nalpha == nbeta");
    const size_t need = sigma_work_layout(ctx, ab_prec, parity, nullptr, nullptr);
    if (need > kScratchBytes)
        return ctx->fail(CASCI_E_UNSUPPORTED, "this string space needs " + std::to_string(need) +
                                                  " bytes of sigma work space, more than the " +
                                                  std::to_string(kScratchBytes) + "-byte static scratch");
    CHECK_RC(need_device(ctx));
    if (!ctx->prepared)
        return ctx->fail(CASCI_E_STATE, "operators not built: run casci_sigma once first (it allocates)");
    unsigned char* base = scratch_addr(ctx->device);
    if (!base) return ctx->fail(CASCI_E_STATE, "no static scratch address for this device");
    DeviceGuard g(ctx->device);
    SigmaWork w;
    sigma_work_layout(ctx, ab_prec, parity, base, &w);
    return sigma_dev(ctx, C, sigma, ab_prec, 0.0, parity, &w);
}

// small device scratch: reduction partials + results
static int ensure_work(casci_ctx* ctx, size_t nout)
{
    HIPC(ctx->d_work.ensure(nout * 512 * 8 + 4096));
    return CASCI_OK;
}

static int dots(casci_ctx* ctx, const double* A, int na, const double* B, int nb, std::vector<double>& out)
{
    const size_t nout = (size_t)na * nb;
    if (nout == 0) {
        out.clear();
        return CASCI_OK;
    }
    CHECK_RC(ensure_work(ctx, nout));
    HIPC(ctx->d_small.ensure(64 * 1024 * 8));
    double* res = ctx->d_small.as<double>() + 49152;  // dedicated region of the scratch block
    if (nout > 16384) return ctx->fail(CASCI_E_ARG, "too many dot products in one call");
    HIPC(launch_block_dot(A, ctx->Nd, na, B, ctx->Nd, nb, ctx->Nd, ctx->d_work.as<double>(), res,
                          ctx->stream));
    out.resize(nout);
    HIPC(hipMemcpyAsync(out.data(), res, nout * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return CASCI_OK;
}

// <S^2> = (Ms^2 + Ms + nb) |C|^2 - <C| sum_pq E^a_qp E^b_pq |C>  (divided by |C|^2)
static int spin_square_dev(casci_ctx* ctx, const double* C, double* s2)
{
    hipStream_t st = ctx->stream;
    const int n = ctx->norb;
    const double ms = 0.5 * (ctx->na - ctx->nb);
    std::vector<double> cc;
    CHECK_RC(dots(ctx, C, 1, C, 1, cc));
    double x = 0.0;
    if (ctx->na > 0 && ctx->nb > 0) {
        if (!ctx->have_s2) {
            std::vector<uint16_t> pairs;
            std::vector<double> vt;
            int M, Mp;
            pair_tables(n, true, pairs, M, Mp);
            build_vt(ctx, pairs, M, Mp, 0.0, 1.0, vt);
            HIPC(ctx->d_pairs_full.ensure(pairs.size() * 2));
            HIPC(ctx->d_vt_s2.ensure(vt.size() * 8));
            HIPC(hipMemcpyAsync(ctx->d_pairs_full.p, pairs.data(), pairs.size() * 2,
                                hipMemcpyHostToDevice, st));
            HIPC(hipMemcpyAsync(ctx->d_vt_s2.p, vt.data(), vt.size() * 8, hipMemcpyHostToDevice, st));
            HIPC(hipStreamSynchronize(st));
            ctx->M_full = M;
            ctx->Mp_full = Mp;
            ctx->have_s2 = true;
        }
        HIPC(ctx->d_t2.ensure((size_t)ctx->Nd * 8));
        HIPC(hipMemsetAsync(ctx->d_t2.p, 0, (size_t)ctx->Nd * 8, st));
        CHECK_RC(ensure_targets(ctx, true));
        AbParams p = ab_params(ctx, true);
        HIPC(ctx->d_rowmax.ensure((size_t)ctx->Na * 8));
        HIPC(launch_row_absmax(C, ctx->Na, ctx->Nb, ctx->d_rowmax.as<double>(), st));
        HIPC(launch_ab_f64(p, ctx->d_vt_s2.as<double>(), C, ctx->d_rowmax.as<double>(), ctx->d_t2.as<double>(), st));
        std::vector<double> cs;
        CHECK_RC(dots(ctx, C, 1, ctx->d_t2.as<double>(), 1, cs));
        x = cs[0];
    }
    *s2 = cc[0] > 0 ? ((ms * ms + ms + ctx->nb) * cc[0] + x) / cc[0] : 0.0;
    return CASCI_OK;
}

extern "C" int casci_spin_square(casci_ctx* ctx, const double* C, double* s2, int mem)
{
    if (!ctx) return CASCI_E_ARG;
    if (!C || !s2) return ctx->fail(CASCI_E_ARG, "C and s2 must not be NULL");
    if (mem != CASCI_MEM_HOST && mem != CASCI_MEM_DEVICE) return ctx->fail(CASCI_E_ARG, "bad mem flag");
    if (!ctx->has_strings) return ctx->fail(CASCI_E_STATE, "build_strings first");
    if (!ctx->has_ints) return ctx->fail(CASCI_E_STATE, "set_integrals first");
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    CHECK_RC(ensure_prepared(ctx, ctx->prepared ? ctx->prepared_lambda : 0.0));
    const double* c = C;
    if (mem == CASCI_MEM_HOST) {
        HIPC(ctx->d_vin.ensure((size_t)ctx->Nd * 8));
        HIPC(hipMemcpyAsync(ctx->d_vin.p, C, (size_t)ctx->Nd * 8, hipMemcpyHostToDevice, ctx->stream));
        c = ctx->d_vin.as<double>();
    }
    return spin_square_dev(ctx, c, s2);
}

// ---------------------------------------------------------------------------
// reduced density matrices
// ---------------------------------------------------------------------------
// g1 (device, 2 n^2) and g2 (device, 3 n^4 or null) of a device vector C: the
// rows M = [D^alpha ; D^beta ; C] of a block of alpha strings (at most 512 MiB)
// are filled on the device and their Gram matrix G = M M^T accumulated block
// by block with a library DGEMM (fixed blocking, so the sums are reproducible),
// then the matrices are read off G (rdm_kernels.hip).
static int rdm_dev(casci_ctx* ctx, const double* C, double* g1, double* g2)
{
    hipStream_t st = ctx->stream;
    const int n = ctx->norb;
    const int64_t R = 2 * (int64_t)n * n + 1;
    const int64_t Na = ctx->Na, Nb = ctx->Nb;
    const int64_t per_alpha = R * Nb * 8;
    int64_t nblk = std::max<int64_t>(1, ((int64_t)512 << 20) / per_alpha);
    nblk = std::min(nblk, Na);
    if (nblk * Nb > 0x7fffffffLL) nblk = std::max<int64_t>(1, 0x7fffffffLL / Nb);
    HIPC(ctx->d_rdm_M.ensure((size_t)(R * nblk * Nb * 8)));
    HIPC(ctx->d_rdm_G.ensure((size_t)(R * R * 8)));
    if (!ctx->blas) {
        if (rocblas_create_handle(&ctx->blas) != rocblas_status_success) {
            ctx->blas = nullptr;
            return ctx->fail(CASCI_E_DEVICE, "rocblas_create_handle failed");
        }
    }
    if (rocblas_set_stream(ctx->blas, st) != rocblas_status_success)
        return ctx->fail(CASCI_E_DEVICE, "rocblas_set_stream failed");
    double* M = ctx->d_rdm_M.as<double>();
    double* G = ctx->d_rdm_G.as<double>();
    const double one = 1.0, zero = 0.0;
    for (int64_t a0 = 0; a0 < Na; a0 += nblk) {
        const int64_t b = std::min(nblk, Na - a0);
        const int64_t ldm = b * Nb;
        HIPC(launch_rdm_fill(C, a0, b, Nb, n, ctx->na, ctx->nb, ctx->d_astr.as<uint64_t>(),
                             ctx->d_bstr.as<uint64_t>(), ctx->d_la_j.as<int32_t>(), ctx->sa,
                             ctx->d_lb_j.as<int32_t>(), ctx->sb, M, ldm, st));
        // G (+)= M M^T: M is the column-major ldm x R matrix A = M^T, G = A^T A
        const rocblas_status s = rocblas_dgemm(ctx->blas, rocblas_operation_transpose, rocblas_operation_none,
                                               (rocblas_int)R, (rocblas_int)R, (rocblas_int)ldm, &one, M,
                                               (rocblas_int)ldm, M, (rocblas_int)ldm, a0 == 0 ? &zero : &one, G,
                                               (rocblas_int)R);
        if (s != rocblas_status_success)
            return ctx->fail(CASCI_E_DEVICE, std::string("rocblas_dgemm: ") + rocblas_status_to_string(s));
    }
    HIPC(launch_rdm_assemble(G, n, g1, g2, st));
    return CASCI_OK;
}

static int rdm_common(casci_ctx* ctx, const double* C, int mem, bool two, bool spin_free, double* o1, double* o2)
{
    if (!ctx) return CASCI_E_ARG;
    if (!C || !o1) return ctx->fail(CASCI_E_ARG, "C and the one-particle output must not be NULL");
    if (mem != CASCI_MEM_HOST && mem != CASCI_MEM_DEVICE) return ctx->fail(CASCI_E_ARG, "bad mem flag");
    if (!ctx->has_strings) return ctx->fail(CASCI_E_STATE, "build_strings first");
    const int n = ctx->norb;
    const size_t n2 = (size_t)n * n, n4 = n2 * n2;
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t st = ctx->stream;
    const double* c = C;
    if (mem == CASCI_MEM_HOST) {
        HIPC(ctx->d_vin.ensure((size_t)ctx->Nd * 8));
        HIPC(hipMemcpyAsync(ctx->d_vin.p, C, (size_t)ctx->Nd * 8, hipMemcpyHostToDevice, st));
        c = ctx->d_vin.as<double>();
    }
    // outputs on the device: spin-resolved g1, g2, then the spin sums
    const size_t nres = 2 * n2 + (two ? 3 * n4 : 0), nsf = spin_free ? n2 + (two ? n4 : 0) : 0;
    HIPC(ctx->d_rdm_out.ensure((nres + nsf) * 8));
    double* g1 = ctx->d_rdm_out.as<double>();
    double* g2 = two ? g1 + 2 * n2 : nullptr;
    CHECK_RC(rdm_dev(ctx, c, g1, g2));
    if (spin_free) {
        double* gam = g1 + nres;
        double* Gam = two ? gam + n2 : nullptr;
        HIPC(launch_rdm_spin_free(g1, g2, n, gam, Gam, st));
        HIPC(hipMemcpyAsync(o1, gam, n2 * 8, hipMemcpyDeviceToHost, st));
        if (two) HIPC(hipMemcpyAsync(o2, Gam, n4 * 8, hipMemcpyDeviceToHost, st));
    } else {
        HIPC(hipMemcpyAsync(o1, g1, 2 * n2 * 8, hipMemcpyDeviceToHost, st));
        if (two) HIPC(hipMemcpyAsync(o2, g2, 3 * n4 * 8, hipMemcpyDeviceToHost, st));
    }
    HIPC(hipStreamSynchronize(st));
    return CASCI_OK;
}

extern "C" int casci_rdm(casci_ctx* ctx, const double* C, int mem, double* g1, double* g2)
{
    return rdm_common(ctx, C, mem, g2 != nullptr, false, g1, g2);
}

extern "C" int casci_rdm_spin_free(casci_ctx* ctx, const double* C, int mem, double* gamma, double* Gamma)
{
    return rdm_common(ctx, C, mem, Gamma != nullptr, true, gamma, Gamma);
}

// ---------------------------------------------------------------------------
// Davidson-Liu
// ---------------------------------------------------------------------------
namespace {

struct Timer {
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    double ms() const
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

}  // namespace

// training-data collector run inside Davidson (casci_mlp_collect)
struct Collector {
    const double* xstar;  // device [nroots][Ndet]
    int samples;
    uint64_t seed;
    float* F;             // device [max_rows][MLP_IN]
    float* T;             // device [max_rows]
    int64_t max_rows;
    int64_t rows = 0;
};

static int davidson_impl(casci_ctx* ctx, int nroots, double tol, const casci_davidson_opts* opts,
                         double* energies, void* vectors, int mem, casci_davidson_info* info,
                         Collector* col);

extern "C" int casci_davidson(casci_ctx* ctx, int nroots, double tol, const casci_davidson_opts* opts,
                              double* energies, void* vectors, int mem, casci_davidson_info* info)
{
    return davidson_impl(ctx, nroots, tol, opts, energies, vectors, mem, info, nullptr);
}

static MlpFeatArgs mlp_args(const casci_ctx* ctx, const double* x, const double* sx, double theta,
                            double rnorm, double dmin)
{
    MlpFeatArgs a;
    a.diag = ctx->d_diag.as<double>();
    a.x = x;
    a.sx = sx;
    a.theta = theta;
    a.rnorm = rnorm;
    a.dmin = dmin;
    a.astr = ctx->d_astr.as<uint64_t>();
    a.bstr = ctx->d_bstr.as<uint64_t>();
    a.N = ctx->Nd;
    a.Nb = ctx->Nb;
    a.n = ctx->norb;
    a.na = ctx->na;
    a.nb = ctx->nb;
    return a;
}

// one iteration of training-data collection: for every root, `samples`
// random determinants get their features and the normalised error x* - x
static int collect_step(casci_ctx* ctx, Collector* col, int k, const double* X, const double* SX,
                        const std::vector<double>& theta, const std::vector<double>& rn, double dmin)
{
    const int64_t Nd = ctx->Nd;
    hipStream_t st = ctx->stream;
    for (int j = 0; j < k && col->rows < col->max_rows; ++j) {
        const double* x = X + (size_t)j * Nd;
        const double* xs = col->xstar + (size_t)j * Nd;
        std::vector<double> d1, d2;
        CHECK_RC(dots(ctx, xs, 1, x, 1, d1));
        CHECK_RC(dots(ctx, xs, 1, xs, 1, d2));
        const double sgn = d1[0] >= 0 ? 1.0 : -1.0;
        const double dn2 = d2[0] + 1.0 - 2.0 * sgn * d1[0];  // |s x* - x|^2 with |x| = 1
        if (!(dn2 > 1e-24)) continue;
        const int m = (int)std::min<int64_t>(col->samples, col->max_rows - col->rows);
        std::vector<int64_t> idx(m);
        uint64_t z = col->seed + 0x9E3779B97F4A7C15ull * (uint64_t)(col->rows + 1);
        for (int i = 0; i < m; ++i) {  // splitmix64 stream
            z += 0x9E3779B97F4A7C15ull;
            uint64_t w = z;
            w = (w ^ (w >> 30)) * 0xBF58476D1CE4E5B9ull;
            w = (w ^ (w >> 27)) * 0x94D049BB133111EBull;
            w ^= w >> 31;
            idx[i] = (int64_t)(w % (uint64_t)Nd);
        }
        HIPC(ctx->d_mlp_idx.ensure((size_t)m * 8));
        HIPC(hipMemcpyAsync(ctx->d_mlp_idx.p, idx.data(), (size_t)m * 8, hipMemcpyHostToDevice, st));
        MlpFeatArgs fa = mlp_args(ctx, x, SX + (size_t)j * Nd, theta[j], rn[j], dmin);
        HIPC(launch_mlp_collect(fa, ctx->d_mlp_idx.as<int64_t>(), m, xs, sgn, 1.0 / std::sqrt(dn2),
                                col->F + col->rows * MLP_IN, col->T + col->rows, st));
        HIPC(hipStreamSynchronize(st));
        col->rows += m;
    }
    return CASCI_OK;
}

// Eigenpairs of a dense symmetric n x n matrix on the host: Householder
// reduction to tridiagonal form with the orthogonal factor formed
// explicitly, then implicit symmetric QR steps with Wilkinson shifts (bulge
// chased by Givens rotations) on the tridiagonal matrix, the rotations
// accumulated into the factor (Golub and Van Loan, Matrix Computations,
// Sec. 5.1 and 8.3). A: row-major, symmetric. w: eigenvalues ascending.
// Z: row-major, column j the unit eigenvector of w[j]. Returns false if the
// QR iteration did not converge.
static bool sym_eig(const double* A, int n, double* w, double* Z)
{
    if (n <= 0) return true;
    std::vector<double> a((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j <= i; ++j) a[(size_t)i * n + j] = a[(size_t)j * n + i] = A[(size_t)i * n + j];
    // reflectors P_k = I - beta_k v_k v_k^T acting on indices k+1..n-1 (v_k[k+1] = 1)
    std::vector<double> vs((size_t)n * n, 0.0), beta(n, 0.0), p(n), wv(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int L = n - k - 1;
        double* v = &vs[(size_t)k * n + k + 1];
        const double x0 = a[(size_t)(k + 1) * n + k];
        double sigma = 0.0;
        for (int i = 1; i < L; ++i) {
            const double xi = a[(size_t)(k + 1 + i) * n + k];
            sigma += xi * xi;
            v[i] = xi;
        }
        v[0] = 1.0;
        double b, mu;
        if (sigma == 0.0) {
            // already reduced in this column (a sign flip is not needed: T may
            // carry a negative off-diagonal)
            beta[k] = 0.0;
            continue;
        }
        mu = std::sqrt(x0 * x0 + sigma);
        const double v0 = x0 <= 0.0 ? x0 - mu : -sigma / (x0 + mu);
        b = 2.0 * v0 * v0 / (sigma + v0 * v0);
        for (int i = 1; i < L; ++i) v[i] /= v0;
        beta[k] = b;
        // trailing block S = a[k+1.., k+1..] <- P S P
        for (int i = 0; i < L; ++i) {
            const double* row = &a[(size_t)(k + 1 + i) * n + k + 1];
            double s = 0.0;
            for (int j = 0; j < L; ++j) s += row[j] * v[j];
            p[i] = b * s;
        }
        double pv = 0.0;
        for (int i = 0; i < L; ++i) pv += p[i] * v[i];
        const double K = 0.5 * b * pv;
        for (int i = 0; i < L; ++i) wv[i] = p[i] - K * v[i];
        for (int i = 0; i < L; ++i) {
            double* row = &a[(size_t)(k + 1 + i) * n + k + 1];
            const double vi = v[i], wi = wv[i];
            for (int j = 0; j < L; ++j) row[j] -= vi * wv[j] + wi * v[j];
        }
        a[(size_t)(k + 1) * n + k] = a[(size_t)k * n + k + 1] = mu;
        for (int i = k + 2; i < n; ++i) a[(size_t)i * n + k] = a[(size_t)k * n + i] = 0.0;
    }
    std::vector<double> d(n), e(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = a[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; ++i) e[i] = a[(size_t)(i + 1) * n + i];
    // Q = P_0 P_1 ... P_{n-3}, stored by columns (zc[j*n + i] = Q[i][j]),
    // accumulated backwards
    std::vector<double> zc((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) zc[(size_t)i * n + i] = 1.0;
    for (int k = n - 3; k >= 0; --k) {
        if (beta[k] == 0.0) continue;
        const double* v = &vs[(size_t)k * n + k + 1];
        const int L = n - k - 1;
        for (int j = k + 1; j < n; ++j) {
            double* q = &zc[(size_t)j * n + k + 1];
            double s = 0.0;
            for (int i = 0; i < L; ++i) s += v[i] * q[i];
            s *= beta[k];
            for (int i = 0; i < L; ++i) q[i] -= s * v[i];
        }
    }
    // implicit symmetric QR on the tridiagonal (d, e)
    const double eps = std::numeric_limits<double>::epsilon();
    int iters = 0;
    const int max_iters = 40 * n + 40;
    int h = n - 1;
    while (h > 0) {
        if (std::fabs(e[h - 1]) <= eps * (std::fabs(d[h - 1]) + std::fabs(d[h])) || e[h - 1] == 0.0) {
            e[h - 1] = 0.0;
            --h;
            continue;
        }
        int l = h - 1;
        while (l > 0 && !(std::fabs(e[l - 1]) <= eps * (std::fabs(d[l - 1]) + std::fabs(d[l])) || e[l - 1] == 0.0))
            --l;
        if (l > 0) e[l - 1] = 0.0;
        if (++iters > max_iters) return false;
        // Wilkinson shift from the trailing 2 x 2 block
        const double dl = 0.5 * (d[h - 1] - d[h]);
        const double eh = e[h - 1];
        const double sg = dl >= 0.0 ? 1.0 : -1.0;
        const double mu = d[h] - eh * eh / (dl + sg * std::hypot(dl, eh));
        double x = d[l] - mu, z = e[l];
        for (int k = l; k < h; ++k) {
            const double r = std::hypot(x, z);
            double c = 1.0, s = 0.0;
            if (r > 0.0) {
                c = x / r;
                s = z / r;
            }
            if (k > l) e[k - 1] = r;
            const double a0 = d[k], b0 = e[k], f0 = d[k + 1];
            d[k] = c * c * a0 + 2.0 * c * s * b0 + s * s * f0;
            d[k + 1] = s * s * a0 - 2.0 * c * s * b0 + c * c * f0;
            e[k] = c * s * (f0 - a0) + (c * c - s * s) * b0;
            if (k + 1 < h) {
                z = s * e[k + 1];
                e[k + 1] *= c;
                x = e[k];
            }
            double* zk = &zc[(size_t)k * n];
            double* zk1 = &zc[(size_t)(k + 1) * n];
            for (int i = 0; i < n; ++i) {
                const double u = zk[i], t = zk1[i];
                zk[i] = c * u + s * t;
                zk1[i] = -s * u + c * t;
            }
        }
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x1, int x2) { return d[x1] < d[x2]; });
    for (int j = 0; j < n; ++j) {
        w[j] = d[ord[j]];
        const double* col = &zc[(size_t)ord[j] * n];
        for (int i = 0; i < n; ++i) Z[(size_t)i * n + j] = col[i];
    }
    return true;
}

// Eigenpairs of the projected matrix G (m x m, row stride ldg). With parity
// (par[i] = +-1 for every basis vector) G is block diagonal and each block is
// solved on its own, so every Ritz vector lies exactly in one parity block;
// the pairs of both blocks are merged in ascending order. theta[0..m), Y
// row-major m x m (column j = eigenvector j).
static bool ritz_eig(const double* G, int ldg, int m, const int* par, bool use_par, double* theta, double* Y)
{
    std::fill(Y, Y + (size_t)m * m, 0.0);
    std::vector<int> blk[2];
    for (int i = 0; i < m; ++i) blk[use_par && par[i] < 0 ? 1 : 0].push_back(i);
    std::vector<std::pair<double, std::pair<int, int>>> all;  // (value, (block, column))
    std::vector<double> wv[2], zv[2];
    for (int b = 0; b < 2; ++b) {
        const int nb = (int)blk[b].size();
        if (nb == 0) continue;
        std::vector<double> Ab((size_t)nb * nb);
        for (int i = 0; i < nb; ++i)
            for (int j = 0; j < nb; ++j) Ab[(size_t)i * nb + j] = G[(size_t)blk[b][i] * ldg + blk[b][j]];
        wv[b].resize(nb);
        zv[b].resize((size_t)nb * nb);
        if (!sym_eig(Ab.data(), nb, wv[b].data(), zv[b].data())) return false;
        for (int j = 0; j < nb; ++j) all.push_back({wv[b][j], {b, j}});
    }
    std::stable_sort(all.begin(), all.end(),
                     [](const std::pair<double, std::pair<int, int>>& x, const std::pair<double, std::pair<int, int>>& y) {
                         return x.first < y.first;
                     });
    for (int j = 0; j < m; ++j) {
        const int b = all[j].second.first, c = all[j].second.second;
        const int nb = (int)blk[b].size();
        theta[j] = all[j].first;
        for (int i = 0; i < nb; ++i) Y[(size_t)blk[b][i] * m + j] = zv[b][(size_t)i * nb + c];
    }
    return true;
}

extern "C" int casci_tile_pairs(int64_t nb, int64_t k0, int64_t count, int64_t* out)
{
    if (nb < 1 || nb > (int64_t)1 << 24 || count < 0 || (count > 0 && !out)) return CASCI_E_ARG;
    const int64_t total = nb * (nb + 1) / 2;
    if (k0 < 0 || k0 + count > total) return CASCI_E_ARG;
    for (int64_t i = 0; i < count; ++i) {
        int64_t bi, bj;
        tile_pair_of(k0 + i, nb, bi, bj);
        out[2 * i] = bi;
        out[2 * i + 1] = bj;
    }
    return CASCI_OK;
}

extern "C" int casci_ss_block_tables(int64_t N, int r, const int32_t* col, const double* val, int R,
                                     int64_t* sizes, uint16_t* uni, int32_t* binfo, uint16_t* goff,
                                     int32_t* rbase, uint32_t* goffs, double* gvals)
{
    if (N < 1 || N >= 65536 || r < 2 || !col || !val || !sizes || (R != SS_BLK_W && R != 2 * SS_BLK_W))
        return CASCI_E_ARG;
    std::vector<int32_t> c(col, col + (size_t)N * r);
    std::vector<double> v(val, val + (size_t)N * r);
    for (int64_t e0 = 0; e0 < N * (int64_t)r; e0 += r)
        for (int e = 1; e < r; ++e) {
            const int32_t J = c[(size_t)e0 + e];
            if (J < 0 || J >= N || (e > 1 && J <= c[(size_t)e0 + e - 1])) return CASCI_E_ARG;
        }
    std::vector<uint16_t> u, go;
    std::vector<int32_t> bi, rb;
    std::vector<SsGroup> g64, g32;
    std::vector<SsGroupF> gf;
    int rc = CASCI_OK;
    const bool ok = build_ss_blocks(N, r, c, v, R, u, go, bi, rb, g64, g32, gf, &rc);
    if (rc != CASCI_OK) return rc;
    if (!ok) {
        for (int i = 0; i < 4; ++i) sizes[i] = 0;
        return CASCI_OK;
    }
    sizes[0] = (int64_t)u.size();
    sizes[1] = (int64_t)g64.size();
    sizes[2] = (int64_t)go.size();
    sizes[3] = (int64_t)(bi.size() / 4);
    if (uni) std::copy(u.begin(), u.end(), uni);
    if (binfo) std::copy(bi.begin(), bi.end(), binfo);
    if (goff) std::copy(go.begin(), go.end(), goff);
    if (rbase) std::copy(rb.begin(), rb.end(), rbase);
    for (size_t i = 0; i < g64.size(); ++i)
        for (int k = 0; k < 4; ++k) {
            if (goffs) goffs[4 * i + k] = g64[i].off[k];
            if (gvals) gvals[4 * i + k] = g64[i].v[k];
        }
    return CASCI_OK;
}

extern "C" int casci_sym_eig(const double* A, int n, double* w, double* Z)
{
    if (n < 0 || (n > 0 && (!A || !w || !Z))) return CASCI_E_ARG;
    for (int64_t i = 0; i < (int64_t)n * n; ++i)
        if (!std::isfinite(A[i])) return CASCI_E_NONFINITE;
    return sym_eig(A, n, w, Z) ? CASCI_OK : CASCI_E_UNSUPPORTED;
}

// Addresses of the `want` lowest entries of d (ties: lower address), ascending:
// one pass with a bounded max-heap, no index array of the full space.
static std::vector<int64_t> lowest_entries(const std::vector<double>& d, int64_t want)
{
    auto less = [&](int64_t a, int64_t b) { return d[a] < d[b] || (d[a] == d[b] && a < b); };
    std::vector<int64_t> heap;
    heap.reserve((size_t)want);
    const int64_t N = (int64_t)d.size();
    for (int64_t i = 0; i < N && want > 0; ++i) {
        if ((int64_t)heap.size() < want) {
            heap.push_back(i);
            std::push_heap(heap.begin(), heap.end(), less);
        } else if (less(i, heap.front())) {
            std::pop_heap(heap.begin(), heap.end(), less);
            heap.back() = i;
            std::push_heap(heap.begin(), heap.end(), less);
        }
    }
    std::sort(heap.begin(), heap.end(), less);
    return heap;
}

// Minimum and maximum of the diagonal (device reduction, fixed partition).
static int diag_range(casci_ctx* ctx, double* lo, double* hi)
{
    DBuf part;
    HIPC(part.ensure(2 * 512 * 8));
    int nblk = 0;
    HIPC(launch_minmax(ctx->d_diag.as<double>(), ctx->Nd, part.as<double>(), &nblk, ctx->stream));
    std::vector<double> h((size_t)2 * nblk);
    HIPC(hipMemcpyAsync(h.data(), part.p, h.size() * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    *lo = INFINITY;
    *hi = -INFINITY;
    for (int b = 0; b < nblk; ++b) {
        *lo = std::fmin(*lo, h[b]);
        *hi = std::fmax(*hi, h[nblk + b]);
    }
    return CASCI_OK;
}

// The `want` lowest diagonal elements (ties: lower address), ascending by
// (value, address): a histogram of the diagonal over [min, max] and the
// entries of the lowest bins that hold at least `want` are found on the
// device; only those are sorted on the host. Bins are monotonic in the value,
// so every entry left out is larger than every one collected and the result
// is exactly that of a full selection. Where the lowest bins hold more than
// 2^22 entries (massively degenerate diagonals) the whole diagonal is
// selected on the host instead.
static int lowest_diag(casci_ctx* ctx, int64_t want, std::vector<int64_t>& out)
{
    out.clear();
    const int64_t Nd = ctx->Nd;
    want = std::min<int64_t>(want, Nd);
    if (want <= 0) return CASCI_OK;
    hipStream_t st = ctx->stream;
    const double* d = ctx->d_diag.as<double>();
    double lo = 0.0, hi = 0.0;
    CHECK_RC(diag_range(ctx, &lo, &hi));
    constexpr int NBINS = 4096;
    constexpr int64_t CAP = (int64_t)1 << 22;
    const double inv_w = hi > lo ? NBINS / (hi - lo) : 0.0;
    DBuf hist, cnt;
    HIPC(hist.ensure(NBINS * 4));
    HIPC(cnt.ensure(8));
    HIPC(hipMemsetAsync(hist.p, 0, NBINS * 4, st));
    HIPC(launch_value_hist(d, Nd, lo, inv_w, NBINS, hist.as<unsigned>(), st));
    std::vector<unsigned> hh(NBINS);
    HIPC(hipMemcpyAsync(hh.data(), hist.p, NBINS * 4, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    int bmax = 0;
    int64_t c = 0;
    for (; bmax < NBINS; ++bmax) {
        c += hh[bmax];
        if (c >= want) break;
    }
    if (bmax == NBINS) return ctx->fail(CASCI_E_DEVICE, "diagonal selection: histogram lost entries");
    auto by_value = [](const std::pair<double, int64_t>& a, const std::pair<double, int64_t>& b) {
        return a.first < b.first || (a.first == b.first && a.second < b.second);
    };
    std::vector<std::pair<double, int64_t>> cand;
    if (c <= CAP) {
        DBuf bidx, bval;
        HIPC(bidx.ensure((size_t)c * 8));
        HIPC(bval.ensure((size_t)c * 8));
        HIPC(hipMemsetAsync(cnt.p, 0, 8, st));
        HIPC(launch_value_collect(d, Nd, lo, inv_w, NBINS, bmax, cnt.as<unsigned long long>(), bidx.as<int64_t>(),
                                  bval.as<double>(), c, st));
        unsigned long long found = 0;
        std::vector<int64_t> h_idx((size_t)c);
        std::vector<double> h_val((size_t)c);
        HIPC(hipMemcpyAsync(&found, cnt.p, 8, hipMemcpyDeviceToHost, st));
        HIPC(hipMemcpyAsync(h_idx.data(), bidx.p, (size_t)c * 8, hipMemcpyDeviceToHost, st));
        HIPC(hipMemcpyAsync(h_val.data(), bval.p, (size_t)c * 8, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        if ((int64_t)found != c) return ctx->fail(CASCI_E_DEVICE, "diagonal selection: histogram and collection disagree");
        cand.resize((size_t)c);
        for (int64_t i = 0; i < c; ++i) cand[(size_t)i] = {h_val[(size_t)i], h_idx[(size_t)i]};
    } else {
        std::vector<double> diag((size_t)Nd);
        HIPC(hipMemcpyAsync(diag.data(), d, (size_t)Nd * 8, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        for (int64_t i : lowest_entries(diag, want)) cand.push_back({diag[(size_t)i], i});
    }
    std::partial_sort(cand.begin(), cand.begin() + want, cand.end(), by_value);
    out.resize((size_t)want);
    for (int64_t i = 0; i < want; ++i) out[(size_t)i] = cand[(size_t)i].second;
    return CASCI_OK;
}

static int davidson_impl(casci_ctx* ctx, int nroots, double tol, const casci_davidson_opts* opts,
                         double* energies, void* vectors, int mem, casci_davidson_info* info,
                         Collector* col)
{
    if (!ctx) return CASCI_E_ARG;
    Timer wall;
    casci_davidson_opts o;
    std::memset(&o, 0, sizeof(o));
    o.ab_prec = CASCI_F64;
    if (opts) o = *opts;
    if (nroots < 1 || nroots > CASCI_MAX_ROOTS) return ctx->fail(CASCI_E_ARG, "nroots must be in [1, 32]");
    if (!(tol > 0.0) || !std::isfinite(tol)) return ctx->fail(CASCI_E_ARG, "tol must be positive");
    if (!energies) return ctx->fail(CASCI_E_ARG, "energies must not be NULL");
    if (mem != CASCI_MEM_HOST && mem != CASCI_MEM_DEVICE) return ctx->fail(CASCI_E_ARG, "bad mem flag");
    if (o.precond != CASCI_PRECOND_DIAG && o.precond != CASCI_PRECOND_OLSEN && o.precond != CASCI_PRECOND_MLP)
        return ctx->fail(CASCI_E_ARG, "unknown preconditioner");
    if (o.spin != CASCI_SPIN_ANY && o.spin != CASCI_SPIN_SINGLET) return ctx->fail(CASCI_E_ARG, "unknown spin target");
    if (o.ab_prec != CASCI_F64 && o.ab_prec != CASCI_F32 && o.ab_prec != CASCI_BF16)
        return ctx->fail(CASCI_E_ARG, "ab_prec must be F64, F32 or BF16");
    if (o.max_iter < 0 || o.m_max < 0) return ctx->fail(CASCI_E_ARG, "negative max_iter or m_max");
    if (!ctx->has_ints) return ctx->fail(CASCI_E_STATE, "set_integrals first");
    if (!ctx->has_strings) return ctx->fail(CASCI_E_STATE, "build_strings first");
    if (o.spin == CASCI_SPIN_SINGLET && ctx->na != ctx->nb)
        return ctx->fail(CASCI_E_ARG, "a singlet target needs nalpha == nbeta");
    const int64_t Nd = ctx->Nd;
    if (nroots > Nd) return ctx->fail(CASCI_E_ARG, "nroots exceeds the number of determinants");
    if (o.guess && o.nguess < nroots) return ctx->fail(CASCI_E_ARG, "need at least nroots guess vectors");
    if (o.guess && o.nguess > 64) return ctx->fail(CASCI_E_ARG, "at most 64 guess vectors");
    if (o.precond == CASCI_PRECOND_MLP && !ctx->have_mlp)
        return ctx->fail(CASCI_E_STATE, "MLP preconditioner selected but no parameters set");
    CHECK_RC(need_device(ctx));
    DeviceGuard guard(ctx->device);

    // nroots requested roots plus buffer roots: Davidson converges the roots it
    // follows, and the highest requested one is easily replaced by a higher
    // state when no root above it is followed
    const int kreq = nroots;
    const int nbuf = o.buffer_roots < 0 ? 0 : (o.buffer_roots == 0 ? 1 : o.buffer_roots);
    const int k = (int)std::min<int64_t>({(int64_t)kreq + nbuf, (int64_t)CASCI_MAX_ROOTS, Nd});
    const int max_iter = o.max_iter > 0 ? o.max_iter : 200;
    int m_max = o.m_max > 0 ? o.m_max : std::max(8, 8 * k);
    m_max = std::min<int64_t>(std::min(m_max, 64), Nd);
    m_max = std::max(m_max, (int)std::min<int64_t>(Nd, 2 * k));
    const double r_tol = o.r_tol > 0 ? o.r_tol : std::max(1e-6, std::sqrt(tol) / 10.0);
    // singlet: lambda S^2 lifts the S = 2, 4, ... states that share the even
    // transposition parity (0 -> 1 Eh; < 0 -> parity only)
    const double lambda = o.spin != CASCI_SPIN_SINGLET ? 0.0
                          : o.s2_penalty > 0         ? o.s2_penalty
                          : o.s2_penalty == 0        ? 1.0
                                                     : 0.0;
    const bool singlet = o.spin == CASCI_SPIN_SINGLET;
    // Mixed precision (ab_prec F32/BF16): sigma of every new correction vector
    // uses the low-precision alpha-beta arithmetic, and at every collapse the
    // sigma of the current Ritz vectors is recomputed in FP64. A correction
    // enters the Ritz vector with a coefficient of the size of the residual,
    // so its sigma error only perturbs the next residual by a relative amount;
    // the refined Ritz vectors carry the FP64 energy. Convergence is declared
    // only on a residual computed from FP64 sigma. `prec` becomes F64 for good
    // if the low-precision phase stalls or the residual drops below
    // refine_rnorm.
    int prec = o.ab_prec;  // alpha-beta arithmetic of new correction vectors
    const double refine_at = o.refine_rnorm > 0 ? o.refine_rnorm : 0.0;

    Timer setup_t;
    CHECK_RC(ensure_prepared(ctx, lambda));
    hipStream_t st = ctx->stream;
    HIPC(hipStreamSynchronize(st));
    const double setup_ms = setup_t.ms();

    // device storage: basis B (m_max + k slots), S (m_max), Ritz X/SX (2k each), temp (1)
    const size_t vb = (size_t)Nd * 8;
    DBuf dB, dS, dX, dSX, dT;
    HIPC(dB.ensure(vb * (m_max + k)));
    HIPC(dS.ensure(vb * (m_max + k)));
    HIPC(dX.ensure(vb * 2 * k));
    HIPC(dSX.ensure(vb * 2 * k));
    HIPC(dT.ensure(vb));
    struct Free {
        DBuf* b[5];
        ~Free()
        {
            for (DBuf* x : b) x->release();
        }
    } free_all{{&dB, &dS, &dX, &dSX, &dT}};
    double* B = dB.as<double>();
    double* S = dS.as<double>();
    double* X = dX.as<double>();
    double* SX = dSX.as<double>();
    auto vB = [&](int i) { return B + (size_t)i * Nd; };
    auto vS = [&](int i) { return S + (size_t)i * Nd; };
    // X and SX hold two sets of k Ritz vectors: the current ones in half `cur`
    // and the previous ones in the other half; a Rayleigh-Ritz step flips the
    // halves instead of copying the previous set
    int cur = 0;
    auto vX = [&](int i) { return X + ((size_t)cur * k + i) * Nd; };
    auto vSX = [&](int i) { return SX + ((size_t)cur * k + i) * Nd; };
    auto vXp = [&](int i) { return X + ((size_t)(1 - cur) * k + i) * Nd; };
    auto vSXp = [&](int i) { return SX + ((size_t)(1 - cur) * k + i) * Nd; };
    HIPC(ctx->d_small.ensure(64 * 1024 * 8));
    double* dsm = ctx->d_small.as<double>();
    // d_small layout (doubles): [8192, 8256) theta, [8320, 8320+4096)
    // coefficients, [32768, ...) reduction results (dots)
    double* dth = dsm + 8192;
    double* dcoef = dsm + 8320;
    double* dres = dsm + 32768;
    CHECK_RC(ensure_work(ctx, 64 * 64));

    hipEvent_t ev0, ev1;
    HIPC(hipEventCreate(&ev0));
    HIPC(hipEventCreate(&ev1));
    struct EvFree {
        hipEvent_t a, b;
        ~EvFree()
        {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } evfree{ev0, ev1};
    double sigma_ms = 0.0;
    int sigma_calls = 0, sigma64 = 0;

    // transposition parity of every basis / Ritz vector (nalpha == nbeta): kept
    // exact by projecting each new vector, so sigma needs one same-spin gather
    const bool use_par = ctx->na == ctx->nb && (singlet || !o.guess);
    std::vector<int> par(m_max + k, 0), xpar(2 * k, 0);
    auto run_sigma_p = [&](const double* c, double* s, int parity, int p) -> int {
        HIPC(hipEventRecord(ev0, st));
        if (o.graph)
            CHECK_RC(sigma_graph(ctx, c, s, p, lambda, use_par ? parity : 0));
        else
            CHECK_RC(sigma_dev(ctx, c, s, p, lambda, use_par ? parity : 0));
        HIPC(hipEventRecord(ev1, st));
        HIPC(hipEventSynchronize(ev1));
        float ms = 0;
        HIPC(hipEventElapsedTime(&ms, ev0, ev1));
        sigma_ms += ms;
        ++sigma_calls;
        if (p == CASCI_F64) ++sigma64;
        return CASCI_OK;
    };
    auto run_sigma = [&](const double* c, double* s, int parity) { return run_sigma_p(c, s, parity, prec); };
    auto dots_dev = [&](const double* A, int na, const double* Bv, int nb, std::vector<double>& out) {
        return dots(ctx, A, na, Bv, nb, out);
    };
    auto combine = [&](const double* A, int na, const std::vector<double>& coef, int nc, double beta,
                       double* Yv) -> int {
        // coef is na x nc row-major
        HIPC(hipMemcpyAsync(dcoef, coef.data(), coef.size() * 8, hipMemcpyHostToDevice, st));
        HIPC(launch_combine(A, Nd, na, dcoef, nc, nc, beta, Yv, Nd, Nd, st));
        HIPC(hipStreamSynchronize(st));  // coef is pageable host memory
        return CASCI_OK;
    };
    auto symmetrize = [&](double* v, int p) -> int {
        // v <- (v + p v^T)/2 for nalpha == nbeta
        HIPC(launch_sym_add(v, ctx->Na, p, 0.5, st));
        return CASCI_OK;
    };
    // the same, with |v|^2 of the result summed in the same pass (per tile
    // pair, then in a fixed order) instead of another pass over v
    auto symmetrize_norm = [&](double* v, int p, double* nrm2) -> int {
        const int64_t parts = sym_add_parts(ctx->Na);
        if (parts > INT32_MAX) return ctx->fail(CASCI_E_UNSUPPORTED, "too many tile pairs for the norm");
        CHECK_RC(ensure_work(ctx, (size_t)(parts + 511) / 512));
        HIPC(launch_sym_add(v, ctx->Na, p, 0.5, st, nullptr, ctx->d_work.as<double>()));
        HIPC(launch_reduce_partials(ctx->d_work.as<double>(), 1, (int)parts, dres, st));
        HIPC(hipMemcpyAsync(nrm2, dres, 8, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        return CASCI_OK;
    };

    // ---- orthonormalise vectors [m, m+cnt) of B against [0, m) and each other;
    // returns the number kept (compacted to [m, m+kept))
    auto orthonormalize = [&](int m, int cnt, int& kept) -> int {
        std::vector<double> c;
        std::vector<double> before(cnt);
        // norms of all new vectors from one Gram-matrix call (its diagonal is
        // summed exactly as a single dot product would be)
        auto norms = [&](std::vector<double>& out) -> int {
            std::vector<double> gram;
            CHECK_RC(dots_dev(vB(m), cnt, vB(m), cnt, gram));
            out.resize(cnt);
            for (int j = 0; j < cnt; ++j) out[j] = std::sqrt(std::max(gram[(size_t)j * cnt + j], 0.0));
            return CASCI_OK;
        };
        CHECK_RC(norms(before));
        std::vector<double> cur = before;  // norms after the Gram-Schmidt against the basis
        if (m > 0) {
            // classical Gram-Schmidt against the basis; the second pass runs only
            // when the first removed most of a vector (norm ratio below 1/sqrt2),
            // which is when one pass can leave a loss of orthogonality
            for (int pass = 0; pass < 2; ++pass) {
                CHECK_RC(dots_dev(vB(0), m, vB(m), cnt, c));
                for (double& x : c) x = -x;
                CHECK_RC(combine(vB(0), m, c, cnt, 1.0, vB(m)));
                if (pass == 0) {
                    CHECK_RC(norms(cur));
                    bool again = false;
                    for (int j = 0; j < cnt; ++j) again = again || !(cur[j] > 0.7071 * before[j]);
                    if (!again) break;
                }
            }
        }
        kept = 0;
        for (int j = 0; j < cnt; ++j) {
            double* v = vB(m + j);
            // Gram-Schmidt against the vectors kept so far. With parity, those of
            // the other parity are orthogonal to v up to rounding: when they all
            // come first (the corrections are generated grouped by parity) only
            // the trailing run of v's parity is used. The second pass runs only
            // when the first removed most of v (the same 1/sqrt2 rule as above,
            // the removed part's norm taken from the coefficients).
            int s0 = 0;
            if (use_par && par[m + j] != 0) {
                s0 = kept;
                while (s0 > 0 && par[m + s0 - 1] == par[m + j]) --s0;
                for (int i = 0; i < s0; ++i)
                    if (par[m + i] == par[m + j] || par[m + i] == 0) s0 = 0;
            }
            if (kept > s0) {
                for (int pass = 0; pass < 2; ++pass) {
                    CHECK_RC(dots_dev(vB(m + s0), kept - s0, v, 1, c));
                    double removed = 0.0;
                    for (double& x : c) {
                        removed += x * x;
                        x = -x;
                    }
                    CHECK_RC(combine(vB(m + s0), kept - s0, c, 1, 1.0, v));
                    if (pass == 0 && !(removed > 0.5 * cur[j] * cur[j])) break;
                }
            }
            // Re-project onto the vector's parity before normalising: what is left
            // after Gram-Schmidt can be small, and normalising it would amplify
            // rounding-level components of the other parity. The projection
            // keeps orthogonality to a basis of pure-parity vectors.
            double n2 = 0.0;
            if (use_par && par[m + j] != 0) {
                CHECK_RC(symmetrize_norm(v, par[m + j], &n2));
            } else {
                std::vector<double> nn;
                CHECK_RC(dots_dev(v, 1, v, 1, nn));
                n2 = nn[0];
            }
            const double nrm = std::sqrt(n2);
            if (!(nrm > 1e-8 * std::max(before[j], 1e-300)) || !(nrm > 1e-14)) continue;
            HIPC(launch_scale(v, 1.0 / nrm, Nd, st));
            if (kept != j) HIPC(hipMemcpyAsync(vB(m + kept), v, vb, hipMemcpyDeviceToDevice, st));
            par[m + kept] = par[m + j];
            ++kept;
        }
        return CASCI_OK;
    };

    std::vector<double> G((size_t)m_max * m_max, 0.0);  // host copy of B^T (H) B, ld = m_max
    // basis vectors [0, nexact) have FP64 sigma: their entries of G are taken
    // as (H b_i)^T b_j, which stays exact when b_j's sigma is low precision
    int nexact = 0;
    auto extend_G = [&](int m0, int cnt) -> int {
        std::vector<double> d, e;
        CHECK_RC(dots_dev(vB(0), m0 + cnt, vS(m0), cnt, d));  // (m0+cnt) x cnt
        const int ne = std::min(nexact, m0 + cnt);
        if (ne > 0 && prec != CASCI_F64) CHECK_RC(dots_dev(vS(0), ne, vB(m0), cnt, e));  // ne x cnt
        for (int i = 0; i < m0 + cnt; ++i)
            for (int j = 0; j < cnt; ++j) {
                const double g = (i < ne && !e.empty()) ? e[(size_t)i * cnt + j] : d[(size_t)i * cnt + j];
                G[(size_t)i * m_max + m0 + j] = g;
                G[(size_t)(m0 + j) * m_max + i] = g;
            }
        return CASCI_OK;
    };

    // ---- initial guess
    int m = 0;
    if (o.guess) {
        const int ng = std::min(o.nguess, m_max);
        HIPC(hipMemcpyAsync(B, o.guess, vb * ng,
                            o.guess_mem == CASCI_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                            st));
        if (singlet)
            for (int j = 0; j < ng; ++j) {
                CHECK_RC(symmetrize(vB(j), 1));
                par[j] = 1;
            }
        int kept = 0;
        CHECK_RC(orthonormalize(0, ng, kept));
        m = kept;
    }
    // the lowest diagonal element (a feature of the learned preconditioner);
    // the start vectors' lowest elements are selected on the device too
    double dmin = 0.0, dmax = 0.0;
    CHECK_RC(diag_range(ctx, &dmin, &dmax));
    if (m < k && !singlet) {
        // Start space: eigenvectors of H in the P-space of the lowest-diagonal
        // determinants (with their transposition partners when nalpha == nbeta,
        // so that both parities are there). Starting from single determinants
        // instead lets Davidson settle on the lowest states of one symmetry
        // and never see a lower state of another.
        const int Pt = (int)std::min<int64_t>(Nd, 240);
        const int64_t want = std::min<int64_t>(Nd, 2 * (int64_t)Pt);
        std::vector<int64_t> idx;
        CHECK_RC(lowest_diag(ctx, want, idx));
        const bool paired = ctx->na == ctx->nb;
        std::vector<int64_t> dets;
        auto has = [&](int64_t x) { return std::find(dets.begin(), dets.end(), x) != dets.end(); };
        for (int64_t t = 0; t < want && (int)dets.size() < Pt; ++t) {
            const int64_t x = idx[t];
            if (has(x)) continue;
            dets.push_back(x);
            if (paired) {
                const int64_t y = (x % ctx->Nb) * ctx->Nb + x / ctx->Nb;
                if (y != x && !has(y)) dets.push_back(y);
            }
        }
        const int P = (int)dets.size();
        DBuf dd, dh;
        HIPC(dd.ensure((size_t)P * 8));
        HIPC(dh.ensure((size_t)P * P * 8));
        HIPC(hipMemcpyAsync(dd.p, dets.data(), (size_t)P * 8, hipMemcpyHostToDevice, st));
        const bool same = ctx->nb == ctx->na;
        HIPC(launch_pspace_h(ctx->norb, P, dd.as<int64_t>(), ctx->Nb, ctx->d_astr.as<uint64_t>(),
                             ctx->d_bstr.as<uint64_t>(), ctx->d_fa_col.as<int32_t>(), ctx->d_fa_val.as<double>(),
                             ctx->ra, (same ? ctx->d_fa_col : ctx->d_fb_col).as<int32_t>(),
                             (same ? ctx->d_fa_val : ctx->d_fb_val).as<double>(), ctx->rb, ctx->d_eri.as<double>(),
                             ctx->d_diag.as<double>(), dh.as<double>(), st));
        std::vector<double> Hp((size_t)P * P), wp, Vp;
        HIPC(hipMemcpyAsync(Hp.data(), dh.p, Hp.size() * 8, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        for (int i = 0; i < P; ++i)  // symmetric by construction up to rounding of the sums
            for (int j = 0; j < i; ++j) Hp[(size_t)i * P + j] = Hp[(size_t)j * P + i];
        wp.resize(P);
        Vp.resize((size_t)P * P);
        if (!sym_eig(Hp.data(), P, wp.data(), Vp.data()))
            return ctx->fail(CASCI_E_UNSUPPORTED, "start space: eigensolver did not converge");
        std::vector<int> partner(P, -1);
        if (paired)
            for (int i = 0; i < P; ++i) {
                const int64_t y = (dets[i] % ctx->Nb) * ctx->Nb + dets[i] / ctx->Nb;
                const auto it2 = std::find(dets.begin(), dets.end(), y);
                partner[i] = it2 == dets.end() ? -1 : (int)(it2 - dets.begin());
            }
        const int nstart = (int)std::min<int64_t>({(int64_t)2 * k, (int64_t)m_max - k, (int64_t)P});
        std::vector<double> y(P);
        for (int j = 0; j < nstart && m < m_max; ++j) {
            double pr = 0.0;
            for (int i = 0; i < P; ++i) {
                y[i] = Vp[(size_t)i * P + j];
                if (partner[i] >= 0) pr += Vp[(size_t)i * P + j] * Vp[(size_t)partner[i] * P + j];
            }
            double* v = vB(m);
            HIPC(hipMemsetAsync(v, 0, vb, st));
            HIPC(hipMemcpyAsync(dh.p, y.data(), (size_t)P * 8, hipMemcpyHostToDevice, st));
            HIPC(launch_scatter_values(dd.as<int64_t>(), dh.as<double>(), P, v, st));
            HIPC(hipStreamSynchronize(st));
            par[m] = paired ? (pr >= 0 ? 1 : -1) : 0;
            if (use_par) CHECK_RC(symmetrize(v, par[m]));
            ++m;
        }
        int kept = 0;
        CHECK_RC(orthonormalize(0, m, kept));
        m = kept;
    }
    if (m < k) {
        // Start vectors from the lowest diagonal elements (ties: lower address).
        // For nalpha == nbeta the determinants (a,b) and (b,a) are combined into
        // (e_ab +- e_ba)/sqrt2: transposition commutes with H and with the
        // diagonal preconditioner, so a space without antisymmetric vectors
        // would never reach odd-S states. SINGLET keeps the + combinations.
        const int64_t want = std::min<int64_t>(Nd, 8 * k + 16);
        std::vector<int64_t> idx;
        CHECK_RC(lowest_diag(ctx, want, idx));

        struct Pick {
            int64_t lo, hi;
            int sign;
        };
        const bool paired = ctx->na == ctx->nb;
        std::vector<Pick> cand;
        auto have = [&](const Pick& c) {
            for (auto& q : cand)
                if (q.lo == c.lo && q.hi == c.hi && q.sign == c.sign) return true;
            return false;
        };
        for (int64_t t = 0; t < want; ++t) {
            const int64_t x = idx[t];
            const int64_t a = x / ctx->Nb, b = x % ctx->Nb;
            const int64_t y = paired ? b * ctx->Nb + a : x;
            Pick ps{std::min(x, y), std::max(x, y), 1};
            if (!have(ps)) cand.push_back(ps);
            if (paired && !singlet && ps.lo != ps.hi) {
                Pick pa{ps.lo, ps.hi, -1};
                if (!have(pa)) cand.push_back(pa);
            }
        }
        // 2k start vectors (at least k+1): Davidson can only converge to states
        // present in the space, and a space of exactly k vectors easily misses one
        const int nstart = std::max(k - m, (int)std::min<int64_t>(
                               {(int64_t)2 * k - m, (int64_t)m_max - k - m, Nd - m}));
        std::vector<Pick> picks;
        for (auto& c : cand)
            if ((int)picks.size() < nstart) picks.push_back(c);
        if (paired && !singlet) {
            bool anti = false;
            for (auto& p : picks) anti |= p.sign < 0;
            if (!anti)
                for (auto& c : cand)
                    if (c.sign < 0) {
                        picks.push_back(c);
                        break;
                    }
        }
        const int start = m;
        for (auto& pr : picks) {
            if (m >= m_max) break;
            double* v = vB(m);
            HIPC(hipMemsetAsync(v, 0, vb, st));
            const double one = 1.0, h2 = std::sqrt(0.5), h2s = pr.sign * std::sqrt(0.5);
            if (pr.lo == pr.hi) {
                HIPC(hipMemcpyAsync(v + pr.lo, &one, 8, hipMemcpyHostToDevice, st));
            } else {
                HIPC(hipMemcpyAsync(v + pr.lo, &h2, 8, hipMemcpyHostToDevice, st));
                HIPC(hipMemcpyAsync(v + pr.hi, &h2s, 8, hipMemcpyHostToDevice, st));
            }
            HIPC(hipStreamSynchronize(st));
            par[m] = pr.sign;
            ++m;
        }
        if (start > 0) {
            int kept = 0;
            CHECK_RC(orthonormalize(start, m - start, kept));
            m = start + kept;
        }
        if (m < k) return ctx->fail(CASCI_E_ARG, "could not build nroots independent start vectors");
    }
    // the start space gets FP64 sigma in every mode: its vectors dominate the
    // first Ritz vectors, and a low-precision error there can reorder nearby
    // states so that a root is lost for good
    for (int j = 0; j < m; ++j) CHECK_RC(run_sigma_p(vB(j), vS(j), par[j], CASCI_F64));
    nexact = m;
    CHECK_RC(extend_G(0, m));

    std::vector<double> theta_prev(k, std::numeric_limits<double>::infinity());
    std::vector<double> theta(64), Y(64 * 64), rn(k, 0.0);
    bool converged = false, have_prev = false;
    int it = 0, switch_iter = -1;
    int empty_steps = 0, mlp_fallbacks = 0, refinements = 0;
    std::vector<double> best_hist;
    for (it = 0; it < max_iter; ++it) {
        // Rayleigh-Ritz (G = B^T H B is kept on the host)
        // With parity, B^T H B is block diagonal (the two parities are orthogonal
        // and H preserves them); its off-block entries are rounding noise and are
        // set to zero, so every Ritz vector lies exactly in one parity block.
        std::vector<double> Gc((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                Gc[(size_t)i * m + j] = (use_par && par[i] != par[j]) ? 0.0 : G[(size_t)i * m_max + j];
        // G is held on the host: its small eigenproblem is solved there
        if (!ritz_eig(Gc.data(), m, m, par.data(), use_par, theta.data(), Y.data()))
            return ctx->fail(CASCI_E_UNSUPPORTED, "Rayleigh-Ritz: eigensolver did not converge");
        // the current Ritz vectors become the previous ones (xpar[k, 2k) holds
        // their parities)
        if (have_prev) {
            cur = 1 - cur;
            for (int j = 0; j < k; ++j) xpar[k + j] = xpar[j];
        }
        // parity of each Ritz vector: the projected matrix is block diagonal in
        // parity, so each eigenvector lives (up to rounding) in one block
        for (int j = 0; j < k; ++j) {
            double wp = 0.0;
            for (int i = 0; i < m; ++i)
                if (par[i] > 0) wp += Y[(size_t)i * m + j] * Y[(size_t)i * m + j];
            xpar[j] = use_par ? (wp >= 0.5 ? 1 : -1) : 0;
        }
        // Ritz vectors X = B Y[:, :k], SX = S Y[:, :k]
        std::vector<double> yk((size_t)m * k);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < k; ++j) yk[(size_t)i * k + j] = Y[(size_t)i * m + j];
        CHECK_RC(combine(vB(0), m, yk, k, 0.0, vX(0)));
        CHECK_RC(combine(vS(0), m, yk, k, 0.0, vSX(0)));
        HIPC(hipMemcpyAsync(dth, theta.data(), k * 8, hipMemcpyHostToDevice, st));
        HIPC(launch_residual(vX(0), vSX(0), Nd, k, dth, ctx->d_diag.as<double>(), Nd, ctx->d_work.as<double>(),
                             dres, st));
        std::vector<double> rs(4 * k);
        HIPC(hipMemcpyAsync(rs.data(), dres, 4 * k * 8, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        double rmax = 0.0;
        std::vector<int> todo;
        for (int j = 0; j < k; ++j) {
            rn[j] = std::sqrt(std::max(rs[4 * j], 0.0));
            if (j < kreq) rmax = std::max(rmax, rn[j]);
            const double dth_j = std::fabs(theta[j] - theta_prev[j]);
            if (j < kreq && !(rn[j] < r_tol && dth_j < tol)) todo.push_back(j);
        }
        // buffer roots get corrections while a requested root is unconverged
        if (!todo.empty())
            for (int j = kreq; j < k; ++j)
                if (!(rn[j] < r_tol && std::fabs(theta[j] - theta_prev[j]) < tol)) todo.push_back(j);
        if (info && info->hist_energy && it < info->hist_len)
            for (int j = 0; j < kreq; ++j) info->hist_energy[(size_t)it * kreq + j] = theta[j];
        if (info && info->hist_residual && it < info->hist_len)
            for (int j = 0; j < kreq; ++j) info->hist_residual[(size_t)it * kreq + j] = rn[j];
        if (info && info->hist_time_ms && it < info->hist_len) info->hist_time_ms[it] = wall.ms();
        for (int j = 0; j < k; ++j) theta_prev[j] = theta[j];
        if (o.progress) o.progress(o.progress_user, it, kreq, theta.data(), rn.data(), wall.ms());
        if (col) CHECK_RC(collect_step(ctx, col, kreq, vX(0), vSX(0), theta, rn, dmin));
        if (!std::isfinite(rmax)) return ctx->fail(CASCI_E_NONFINITE, "non-finite residual in Davidson");
        // collapse: keep current and previous Ritz vectors (room for ncorr new ones)
        auto collapse = [&](int ncorr) -> int {
            const int nkeep = (have_prev && 2 * k + ncorr <= m_max) ? 2 * k : k;
            const bool refine = prec != CASCI_F64;
            HIPC(hipMemcpyAsync(vB(0), vX(0), vb * k, hipMemcpyDeviceToDevice, st));
            HIPC(hipMemcpyAsync(vS(0), vSX(0), vb * k, hipMemcpyDeviceToDevice, st));
            if (nkeep > k) {
                HIPC(hipMemcpyAsync(vB(k), vXp(0), vb * k, hipMemcpyDeviceToDevice, st));
                HIPC(hipMemcpyAsync(vS(k), vSXp(0), vb * k, hipMemcpyDeviceToDevice, st));
            }
            for (int j = 0; j < nkeep; ++j) par[j] = xpar[j];
            if (refine) {  // FP64 sigma of the current Ritz vectors, buffer roots included
                // (refining those in low precision was measured to cost iterations)
                for (int j = 0; j < k; ++j) CHECK_RC(run_sigma_p(vB(j), vS(j), par[j], CASCI_F64));
                ++refinements;
            }
            // Gram-Schmidt of the previous Ritz vectors against the current ones,
            // the same combination applied to their sigma vectors
            int mm = k;
            for (int j = k; j < nkeep; ++j) {
                std::vector<double> c;
                for (int pass = 0; pass < 2; ++pass) {
                    CHECK_RC(dots_dev(vB(0), mm, vB(j), 1, c));
                    for (double& x : c) x = -x;
                    CHECK_RC(combine(vB(0), mm, c, 1, 1.0, vB(j)));
                    CHECK_RC(combine(vS(0), mm, c, 1, 1.0, vS(j)));
                }
                std::vector<double> nn;
                CHECK_RC(dots_dev(vB(j), 1, vB(j), 1, nn));
                const double nrm = std::sqrt(nn[0]);
                // a nearly dependent previous Ritz vector is dropped: normalising a
                // small remainder would amplify rounding (and, with parity, its
                // other-parity part, which its sigma vector does not follow)
                if (nrm < 1e-4) continue;
                HIPC(launch_scale(vB(j), 1.0 / nrm, Nd, st));
                HIPC(launch_scale(vS(j), 1.0 / nrm, Nd, st));
                if (mm != j) {
                    HIPC(hipMemcpyAsync(vB(mm), vB(j), vb, hipMemcpyDeviceToDevice, st));
                    HIPC(hipMemcpyAsync(vS(mm), vS(j), vb, hipMemcpyDeviceToDevice, st));
                }
                par[mm] = par[j];
                // in mixed mode the combined sigma of this small remainder would
                // carry the accumulated low-precision error, amplified by the
                // normalisation: recompute it instead
                if (refine) CHECK_RC(run_sigma(vB(mm), vS(mm), par[mm]));
                ++mm;
            }
            m = mm;
            nexact = refine ? k : m;
            std::fill(G.begin(), G.end(), 0.0);
            CHECK_RC(extend_G(0, m));
            return CASCI_OK;
        };
        // the Ritz data is exact when every vector with a nonzero coefficient
        // has FP64 sigma (always in FP64 mode; in mixed mode right after a
        // refinement that kept only the Ritz vectors)
        const bool exact_now = prec == CASCI_F64 || nexact >= m;
        if (todo.empty() && exact_now) {
            converged = true;
            break;
        }
        if (prec != CASCI_F64) {
            // stalled low-precision phase (no 2x gain of the best residual over
            // 40 iterations), or the optional threshold: FP64 from here on
            best_hist.push_back(rmax);
            const int nh = (int)best_hist.size();
            bool stalled = false;
            if (nh > 80) {
                double recent = *std::min_element(best_hist.end() - 40, best_hist.end());
                double before = *std::min_element(best_hist.begin(), best_hist.end() - 40);
                stalled = recent > 0.5 * before;
            }
            const bool to_f64 = stalled || (refine_at > 0 && rmax < refine_at);
            if (to_f64) {
                // FP64 from here on: restart from the Ritz vectors
                prec = CASCI_F64;
                switch_iter = it;
                HIPC(hipMemcpyAsync(vB(0), vX(0), vb * k, hipMemcpyDeviceToDevice, st));
                for (int j = 0; j < k; ++j) par[j] = xpar[j];
                int kept = 0;
                CHECK_RC(orthonormalize(0, k, kept));
                m = kept;
                for (int j = 0; j < m; ++j) CHECK_RC(run_sigma_p(vB(j), vS(j), par[j], CASCI_F64));
                nexact = m;
                ++refinements;
                std::fill(G.begin(), G.end(), 0.0);
                CHECK_RC(extend_G(0, m));
                have_prev = false;
                for (int j = 0; j < k; ++j) theta_prev[j] = std::numeric_limits<double>::infinity();
                continue;
            }
            if (todo.empty()) {
                // converged on low-precision data: collapse with FP64 sigma of the
                // Ritz vectors and test their exact Rayleigh quotients and residuals
                CHECK_RC(collapse(0));
                std::vector<double> th(k);
                for (int j = 0; j < k; ++j) th[j] = G[(size_t)j * m_max + j];
                HIPC(hipMemcpyAsync(dth, th.data(), k * 8, hipMemcpyHostToDevice, st));
                HIPC(launch_residual(B, S, Nd, k, dth, ctx->d_diag.as<double>(), Nd, ctx->d_work.as<double>(),
                                     dres, st));
                std::vector<double> rx(4 * k);
                HIPC(hipMemcpyAsync(rx.data(), dres, 4 * k * 8, hipMemcpyDeviceToHost, st));
                HIPC(hipStreamSynchronize(st));
                bool ok = true;
                for (int j = 0; j < k; ++j) {
                    const double r = std::sqrt(std::max(rx[4 * j], 0.0));
                    if (j < kreq) ok = ok && r < r_tol && std::fabs(th[j] - theta[j]) < tol;
                    rn[j] = r;
                }
                if (ok) {
                    HIPC(hipMemcpyAsync(vX(0), vB(0), vb * k, hipMemcpyDeviceToDevice, st));
                    for (int j = 0; j < k; ++j) theta[j] = th[j];
                    converged = true;
                    break;
                }
                continue;
            }
        }
        if (m + (int)todo.size() > m_max) CHECK_RC(collapse((int)todo.size()));
        // corrections for unconverged roots, grouped by parity (Gram-Schmidt
        // among the new vectors then skips the other parity)
        if (use_par)
            std::stable_sort(todo.begin(), todo.end(), [&](int a, int b) { return xpar[a] > xpar[b]; });
        const int cnt = (int)todo.size();
        for (int t = 0; t < cnt; ++t) {
            const int j = todo[t];
            double eps = 0.0;
            if (o.precond == CASCI_PRECOND_OLSEN && std::fabs(rs[4 * j + 2]) > 1e-300)
                eps = rs[4 * j + 1] / rs[4 * j + 2];
            bool done = false;
            if (o.precond == CASCI_PRECOND_MLP) {
                MlpFeatArgs fa = mlp_args(ctx, vX(j), vSX(j), theta[j], rn[j], dmin);
                HIPC(launch_mlp_correction(fa, ctx->d_mlp.as<float>(), vB(m + t), st));
                std::vector<double> nn;
                CHECK_RC(dots_dev(vB(m + t), 1, vB(m + t), 1, nn));
                // fallback: a non-finite or vanishing learned correction is replaced by Olsen
                done = std::isfinite(nn[0]) && nn[0] > 0.0;
                if (!done) ++mlp_fallbacks;
            }
            if (!done) {
                if (o.precond == CASCI_PRECOND_MLP && std::fabs(rs[4 * j + 2]) > 1e-300)
                    eps = rs[4 * j + 1] / rs[4 * j + 2];
                HIPC(launch_precondition(vX(j), vSX(j), theta[j], eps, ctx->d_diag.as<double>(), Nd, vB(m + t),
                                         st));
            }
            par[m + t] = xpar[j];
            // Olsen and diagonal corrections of a parity-pure Ritz pair have its
            // parity up to the rounding of H_II, which the re-projection in
            // orthonormalize removes; a learned correction is projected here
            if (use_par && o.precond == CASCI_PRECOND_MLP) CHECK_RC(symmetrize(vB(m + t), xpar[j]));
        }
        int kept = 0;
        CHECK_RC(orthonormalize(m, cnt, kept));
        if (kept == 0) {
            // no new direction (e.g. the subspace already spans the space): one more
            // Rayleigh-Ritz step settles the energy change; a second empty step stops
            if (++empty_steps >= 2) break;
            continue;
        }
        empty_steps = 0;
        for (int j = 0; j < kept; ++j) CHECK_RC(run_sigma(vB(m + j), vS(m + j), par[m + j]));
        if (prec == CASCI_F64) nexact = m + kept;
        CHECK_RC(extend_G(m, kept));
        m += kept;
        have_prev = true;
    }

    // results
    for (int j = 0; j < kreq; ++j) energies[j] = theta[j];
    std::vector<double> s2v(kreq, 0.0);
    if (vectors || info) {
        for (int j = 0; j < kreq; ++j) {
            // phase: largest-|c| entry positive (ties: lowest index), found on the device
            double am[2];
            HIPC(launch_absmax(vX(j), Nd, ctx->d_work.as<double>(), dres, st));
            HIPC(hipMemcpyAsync(am, dres, sizeof(am), hipMemcpyDeviceToHost, st));
            HIPC(hipStreamSynchronize(st));
            if (am[0] < 0) HIPC(launch_scale(vX(j), -1.0, Nd, st));
            if (info) CHECK_RC(spin_square_dev(ctx, vX(j), &s2v[j]));
        }
        if (vectors)
            HIPC(hipMemcpyAsync(vectors, vX(0), vb * kreq,
                                mem == CASCI_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, st));
        HIPC(hipStreamSynchronize(st));
    }
    if (info) {
        info->iterations = it + (converged ? 1 : 0);
        info->sigma_calls = sigma_calls;
        info->sigma_calls_fp64 = sigma64;
        info->converged = converged ? 1 : 0;
        info->switch_iter = switch_iter < 0 ? -1 : switch_iter;
        info->mlp_fallbacks = mlp_fallbacks;
        info->refinements = refinements;
        for (int j = 0; j < CASCI_MAX_ROOTS; ++j) {
            info->residual[j] = j < kreq ? rn[j] : 0.0;
            info->s2[j] = j < kreq ? s2v[j] : 0.0;
        }
        info->time_sigma_ms = sigma_ms;
        info->time_setup_ms = setup_ms;
        info->time_total_ms = wall.ms();
    }
    return converged ? CASCI_OK : CASCI_NOCONV;
}

// ---------------------------------------------------------------------------
// learned preconditioner
// ---------------------------------------------------------------------------
static int mlp_upload(casci_ctx* ctx, const float* src, size_t n, int mem, DBuf& dst)
{
    HIPC(dst.ensure(n * 4));
    HIPC(hipMemcpyAsync(dst.p, src, n * 4, mem == CASCI_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                        ctx->stream));
    if (mem == CASCI_MEM_HOST) HIPC(hipStreamSynchronize(ctx->stream));
    return CASCI_OK;
}

extern "C" int casci_mlp_set_params(casci_ctx* ctx, const float* params, int64_t n, int mem)
{
    if (!ctx) return CASCI_E_ARG;
    if (!params) return ctx->fail(CASCI_E_ARG, "params is NULL");
    if (n != MLP_NPARAM) return ctx->fail(CASCI_E_ARG, "expected MLP_NPARAM parameters");
    if (mem != CASCI_MEM_HOST && mem != CASCI_MEM_DEVICE) return ctx->fail(CASCI_E_ARG, "bad mem flag");
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    CHECK_RC(mlp_upload(ctx, params, MLP_NPARAM, mem, ctx->d_mlp));
    HIPC(ctx->d_mlp_m.ensure(MLP_NPARAM * 4));
    HIPC(ctx->d_mlp_v.ensure(MLP_NPARAM * 4));
    HIPC(hipMemsetAsync(ctx->d_mlp_m.p, 0, MLP_NPARAM * 4, ctx->stream));
    HIPC(hipMemsetAsync(ctx->d_mlp_v.p, 0, MLP_NPARAM * 4, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    ctx->have_mlp = true;
    return CASCI_OK;
}

extern "C" int casci_mlp_get_params(casci_ctx* ctx, float* out)
{
    if (!ctx) return CASCI_E_ARG;
    if (!out) return ctx->fail(CASCI_E_ARG, "out is NULL");
    if (!ctx->have_mlp) return ctx->fail(CASCI_E_STATE, "no MLP parameters set");
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    HIPC(hipMemcpyAsync(out, ctx->d_mlp.p, MLP_NPARAM * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return CASCI_OK;
}

extern "C" int casci_mlp_forward(casci_ctx* ctx, const float* X, int64_t N, float* Y, int mem)
{
    if (!ctx) return CASCI_E_ARG;
    if (!X || !Y || N < 0) return ctx->fail(CASCI_E_ARG, "bad arguments");
    if (mem != CASCI_MEM_HOST && mem != CASCI_MEM_DEVICE) return ctx->fail(CASCI_E_ARG, "bad mem flag");
    if (!ctx->have_mlp) return ctx->fail(CASCI_E_STATE, "no MLP parameters set");
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t st = ctx->stream;
    const float* dx = X;
    float* dy = Y;
    DBuf bx, by;
    if (mem == CASCI_MEM_HOST) {
        HIPC(bx.ensure((size_t)N * MLP_IN * 4 + 16));
        HIPC(by.ensure((size_t)N * 4 + 16));
        HIPC(hipMemcpyAsync(bx.p, X, (size_t)N * MLP_IN * 4, hipMemcpyHostToDevice, st));
        dx = bx.as<float>();
        dy = by.as<float>();
    }
    HIPC(launch_mlp_forward(ctx->d_mlp.as<float>(), dx, N, dy, st));
    if (mem == CASCI_MEM_HOST) {
        HIPC(hipMemcpyAsync(Y, dy, (size_t)N * 4, hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        bx.release();
        by.release();
    }
    return CASCI_OK;
}

// gradient of the mean squared error over all N samples with the current params
static int mlp_grad_full(casci_ctx* ctx, const float* dX, const float* dT, int64_t N, const int32_t* perm,
                         int64_t begin, int64_t count, double* sse)
{
    const int nblocks = 512;
    HIPC(ctx->d_mlp_part.ensure((size_t)nblocks * (MLP_NPARAM + 1) * 4));
    HIPC(ctx->d_mlp_g.ensure(MLP_NPARAM * 4));
    HIPC(ctx->d_mlp_sse.ensure(64));
    HIPC(launch_mlp_grad(ctx->d_mlp.as<float>(), dX, dT, perm, begin, count, count,
                         ctx->d_mlp_part.as<float>(), nblocks, ctx->d_mlp_g.as<float>(),
                         ctx->d_mlp_sse.as<double>(), ctx->stream));
    (void)N;
    if (sse) {
        HIPC(hipMemcpyAsync(sse, ctx->d_mlp_sse.p, 8, hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
    }
    return CASCI_OK;
}

static int mlp_stage(casci_ctx* ctx, const float* X, const float* T, int64_t N, int mem, DBuf& bx, DBuf& bt,
                     const float** dX, const float** dT)
{
    *dX = X;
    *dT = T;
    if (mem == CASCI_MEM_HOST) {
        HIPC(bx.ensure((size_t)N * MLP_IN * 4 + 16));
        HIPC(bt.ensure((size_t)N * 4 + 16));
        HIPC(hipMemcpyAsync(bx.p, X, (size_t)N * MLP_IN * 4, hipMemcpyHostToDevice, ctx->stream));
        HIPC(hipMemcpyAsync(bt.p, T, (size_t)N * 4, hipMemcpyHostToDevice, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
        *dX = bx.as<float>();
        *dT = bt.as<float>();
    }
    return CASCI_OK;
}

static int mlp_identity_perm(casci_ctx* ctx, int64_t N)
{
    std::vector<int32_t> perm(N);
    for (int64_t i = 0; i < N; ++i) perm[i] = (int32_t)i;
    HIPC(ctx->d_mlp_perm.ensure((size_t)N * 4 + 16));
    HIPC(hipMemcpyAsync(ctx->d_mlp_perm.p, perm.data(), (size_t)N * 4, hipMemcpyHostToDevice, ctx->stream));
    HIPC(hipStreamSynchronize(ctx->stream));
    return CASCI_OK;
}

extern "C" int casci_mlp_loss_grad(casci_ctx* ctx, const float* X, const float* T, int64_t N, float* grad,
                                   double* loss, int mem)
{
    if (!ctx) return CASCI_E_ARG;
    if (!X || !T || N <= 0 || N >= (1LL << 31)) return ctx->fail(CASCI_E_ARG, "bad arguments");
    if (mem != CASCI_MEM_HOST && mem != CASCI_MEM_DEVICE) return ctx->fail(CASCI_E_ARG, "bad mem flag");
    if (!ctx->have_mlp) return ctx->fail(CASCI_E_STATE, "no MLP parameters set");
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    DBuf bx, bt;
    const float *dX, *dT;
    CHECK_RC(mlp_stage(ctx, X, T, N, mem, bx, bt, &dX, &dT));
    CHECK_RC(mlp_identity_perm(ctx, N));
    double sse = 0.0;
    CHECK_RC(mlp_grad_full(ctx, dX, dT, N, ctx->d_mlp_perm.as<int32_t>(), 0, N, &sse));
    if (loss) *loss = sse / (double)N;
    if (grad) {
        HIPC(hipMemcpyAsync(grad, ctx->d_mlp_g.p, MLP_NPARAM * 4, hipMemcpyDeviceToHost, ctx->stream));
        HIPC(hipStreamSynchronize(ctx->stream));
    }
    bx.release();
    bt.release();
    return CASCI_OK;
}

extern "C" int casci_mlp_train(casci_ctx* ctx, const float* X, const float* T, int64_t N, int epochs,
                               int batch, float lr, uint64_t seed, double* loss_hist, int mem)
{
    if (!ctx) return CASCI_E_ARG;
    if (!X || !T || N <= 0 || N >= (1LL << 31) || epochs < 1 || batch < 64 || !(lr > 0))
        return ctx->fail(CASCI_E_ARG, "bad arguments");
    if (mem != CASCI_MEM_HOST && mem != CASCI_MEM_DEVICE) return ctx->fail(CASCI_E_ARG, "bad mem flag");
    if (!ctx->have_mlp) return ctx->fail(CASCI_E_STATE, "set initial MLP parameters first");
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    hipStream_t st = ctx->stream;
    DBuf bx, bt;
    const float *dX, *dT;
    CHECK_RC(mlp_stage(ctx, X, T, N, mem, bx, bt, &dX, &dT));
    std::vector<int32_t> perm(N);
    for (int64_t i = 0; i < N; ++i) perm[i] = (int32_t)i;
    HIPC(ctx->d_mlp_perm.ensure((size_t)N * 4 + 16));
    uint64_t z = seed;
    int step = 0;
    for (int ep = 0; ep < epochs; ++ep) {
        for (int64_t i = N - 1; i > 0; --i) {  // Fisher-Yates with splitmix64
            z += 0x9E3779B97F4A7C15ull;
            uint64_t w = z;
            w = (w ^ (w >> 30)) * 0xBF58476D1CE4E5B9ull;
            w = (w ^ (w >> 27)) * 0x94D049BB133111EBull;
            w ^= w >> 31;
            std::swap(perm[i], perm[w % (uint64_t)(i + 1)]);
        }
        HIPC(hipMemcpyAsync(ctx->d_mlp_perm.p, perm.data(), (size_t)N * 4, hipMemcpyHostToDevice, st));
        HIPC(hipStreamSynchronize(st));
        double ep_sse = 0.0;
        for (int64_t b0 = 0; b0 < N; b0 += batch) {
            const int64_t cnt = std::min<int64_t>(batch, N - b0);
            double sse = 0.0;
            CHECK_RC(mlp_grad_full(ctx, dX, dT, N, ctx->d_mlp_perm.as<int32_t>(), b0, cnt, &sse));
            ep_sse += sse;
            HIPC(launch_adam(ctx->d_mlp.as<float>(), ctx->d_mlp_g.as<float>(), ctx->d_mlp_m.as<float>(),
                             ctx->d_mlp_v.as<float>(), lr, ++step, st));
        }
        if (loss_hist) loss_hist[ep] = ep_sse / (double)N;
    }
    HIPC(hipStreamSynchronize(st));
    bx.release();
    bt.release();
    return CASCI_OK;
}

extern "C" int casci_mlp_collect(casci_ctx* ctx, int nroots, double tol, const casci_davidson_opts* opts,
                                 const double* xstar, int samples, uint64_t seed, float* F, float* T,
                                 int64_t max_rows, int64_t* nrows)
{
    if (!ctx) return CASCI_E_ARG;
    if (!xstar || !F || !T || !nrows || samples < 1 || max_rows < 1)
        return ctx->fail(CASCI_E_ARG, "bad arguments");
    Collector col;
    col.xstar = xstar;
    col.samples = samples;
    col.seed = seed;
    col.F = F;
    col.T = T;
    col.max_rows = max_rows;
    std::vector<double> E(nroots > 0 && nroots <= CASCI_MAX_ROOTS ? nroots : 1);
    const int rc = davidson_impl(ctx, nroots, tol, opts, E.data(), nullptr, CASCI_MEM_HOST, nullptr, &col);
    *nrows = col.rows;
    return rc;
}

extern "C" int casci_mlp_features(casci_ctx* ctx, const double* x, const double* sx, double theta,
                                  const int64_t* idx, int m, float* F)
{
    if (!ctx) return CASCI_E_ARG;
    if (!x || !sx || !idx || !F || m < 0) return ctx->fail(CASCI_E_ARG, "bad arguments");
    if (!ctx->has_ints) return ctx->fail(CASCI_E_STATE, "set_integrals first");
    if (!ctx->has_strings) return ctx->fail(CASCI_E_STATE, "build_strings first");
    for (int i = 0; i < m; ++i)
        if (idx[i] < 0 || idx[i] >= ctx->Nd) return ctx->fail(CASCI_E_ARG, "determinant index out of range");
    CHECK_RC(need_device(ctx));
    DeviceGuard g(ctx->device);
    CHECK_RC(ensure_prepared(ctx, ctx->prepared ? ctx->prepared_lambda : 0.0));
    hipStream_t st = ctx->stream;
    const size_t vb = (size_t)ctx->Nd * 8;
    std::vector<double> diag(ctx->Nd);
    HIPC(hipMemcpyAsync(diag.data(), ctx->d_diag.p, vb, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    const double dmin = *std::min_element(diag.begin(), diag.end());
    // residual norm |sx - theta x| from two dots and the cross term
    std::vector<double> xx, ss, xs;
    CHECK_RC(dots(ctx, x, 1, x, 1, xx));
    CHECK_RC(dots(ctx, sx, 1, sx, 1, ss));
    CHECK_RC(dots(ctx, x, 1, sx, 1, xs));
    const double rn = std::sqrt(std::max(0.0, ss[0] - 2 * theta * xs[0] + theta * theta * xx[0]));
    HIPC(ctx->d_mlp_idx.ensure((size_t)m * 8 + 8));
    HIPC(hipMemcpyAsync(ctx->d_mlp_idx.p, idx, (size_t)m * 8, hipMemcpyHostToDevice, st));
    DBuf bf;
    HIPC(bf.ensure((size_t)m * MLP_IN * 4 + 16));
    MlpFeatArgs fa = mlp_args(ctx, x, sx, theta, rn, dmin);
    HIPC(launch_mlp_collect(fa, ctx->d_mlp_idx.as<int64_t>(), m, nullptr, 1.0, 0.0, bf.as<float>(), nullptr, st));
    HIPC(hipMemcpyAsync(F, bf.p, (size_t)m * MLP_IN * 4, hipMemcpyDeviceToHost, st));
    HIPC(hipStreamSynchronize(st));
    bf.release();
    return CASCI_OK;
}

extern "C" int casci_batch_davidson(casci_ctx* const* ctxs, int count, int nroots, double tol,
                                    const casci_davidson_opts* opts, double* energies,
                                    casci_davidson_info* infos, int nthreads)
{
    if (!ctxs || count < 0 || (count > 0 && !energies)) return CASCI_E_ARG;
    for (int i = 0; i < count; ++i) {
        if (!ctxs[i]) return CASCI_E_ARG;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return ctxs[i]->fail(CASCI_E_ARG, "a context appears twice in the batch");
    }
    if (count == 0) return CASCI_OK;
    int nt = nthreads > 0 ? nthreads : 16;
    nt = std::max(1, std::min(nt, count));
    std::atomic<int> next(0);
    std::vector<int> rc(count, CASCI_OK);
    auto worker = [&]() {
        for (;;) {
            const int i = next.fetch_add(1);
            if (i >= count) break;
            rc[i] = davidson_impl(ctxs[i], nroots, tol, opts, energies + (size_t)i * nroots, nullptr,
                                  CASCI_MEM_HOST, infos ? infos + i : nullptr, nullptr);
        }
    };
    std::vector<std::thread> pool;
    pool.reserve(nt - 1);
    for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
    worker();
    for (auto& th : pool) th.join();
    int out = CASCI_OK;
    for (int i = 0; i < count; ++i)
        if (rc[i] < 0) return rc[i];
        else if (rc[i] > 0) out = rc[i];
    return out;
}

