// The residual F = A Phi + [N(u); 0; 0] - b (eq. general_nonlinear) for
// callers that cannot allocate device memory (code under HIP graph capture,
// tight serving loops): the same kernels as pbfb_residual, with every work
// buffer carved from one file-scope device array instead of the problem's
// scratch.  The array exists once per device (held until the process ends);
// its device address is taken once per device, with that device current,
// when a context is created there, and only that address is ever handed to
// kernels or copies.
#include <mutex>

#include "pbfb_internal.hpp"

// the work array (global namespace: the library's own pbfb::scratch helper
// is a different thing)
static __device__ __align__(256) unsigned char scratch[size_t(256) << 20];

namespace pbfb {

constexpr size_t NOALLOC_BYTES = sizeof(::scratch); // 256 MiB per device
constexpr int NOALLOC_MAX_DEVICES = 64;

static std::mutex g_noalloc_mu;
static void *g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// called by pbfb_ctx_create with `device` current
void noalloc_init(int device)
{
    PB_CHECK(device >= 0 && device < NOALLOC_MAX_DEVICES, PBFB_EINVAL, "device id out of range");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (g_noalloc_ptr[device]) return;
    void *ptr = nullptr;
    PB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(::scratch)));
    PB_CHECK(ptr != nullptr, PBFB_EDEVICE, "no device address for the residual work array");
    g_noalloc_ptr[device] = ptr;
}

static void *noalloc_base(int device)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    return device >= 0 && device < NOALLOC_MAX_DEVICES ? g_noalloc_ptr[device] : nullptr;
}

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// Work bytes of one residual: N(u) on the FEM rows, 4 element terms per tet,
// the packed surface inputs, and (when a surface is stored symmetric, which
// is assumed here so that the bound holds before setup) its column partials.
size_t noalloc_residual_bytes(const Problem &p)
{
    size_t b = round256(sizeof(double) * size_t(p.nn)) + round256(sizeof(double) * 4 * size_t(p.ntet));
    for (int w = 0; w < 2; ++w) {
        const int64_t nv = p.topo[w].nv;
        b += round256(sizeof(double) * size_t(bem_ld(nv))) + round256(sizeof(double) * size_t(sym_partials_doubles(nv)));
    }
    return b;
}

} // namespace pbfb

using namespace pbfb;

extern "C" pbfb_status pbfb_residual_noalloc(pbfb_problem *pp, int scheme, const double *phi, double *F,
                                             void *hip_stream)
{
    try {
        PB_CHECK(pp && phi && F, PBFB_EINVAL, "null argument");
        PB_CHECK(scheme >= PBFB_LIN && scheme <= PBFB_T7, PBFB_EINVAL, "unknown scheme");
        Problem &p = pp->p;
        PB_CHECK(p.ctx, PBFB_ESTATE, "the problem's context was destroyed");
        PB_CHECK(p.have_mesh, PBFB_ESTATE, "set_mesh must precede the residual");
        const size_t need = noalloc_residual_bytes(p);
        PB_CHECK(need <= NOALLOC_BYTES, PBFB_EINVAL,
                 "problem too large for the allocation-free residual: it needs " + std::to_string(need) +
                     " bytes of work memory, the limit is " + std::to_string(NOALLOC_BYTES));
        PB_CHECK(!p.bem_mf, PBFB_EINVAL, "the allocation-free residual needs stored (dense) boundary operators");
        PB_CHECK(p.topo_ready && p.geom_ready && p.val_ready && p.fm_ready && p.bem_ready[0] && p.bem_ready[1],
                 PBFB_ESTATE, "the problem is not set up (call pbfb_setup first)");
        for (const void *v : {static_cast<const void *>(phi), static_cast<const void *>(F)}) {
            hipPointerAttribute_t at{};
            PB_CHECK(hipPointerGetAttributes(&at, v) == hipSuccess && at.type == hipMemoryTypeDevice &&
                         at.device == p.ctx->device,
                     PBFB_EINVAL, "phi and F must be device memory of the context's GPU");
        }
        hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : p.ctx->stream;
        PB_HIP(hipSetDevice(p.ctx->device));
        unsigned char *base = static_cast<unsigned char *>(noalloc_base(p.ctx->device));
        PB_CHECK(base, PBFB_ESTATE, "no context was created on this device");
        size_t off = 0;
        auto take = [&](size_t n) {
            double *d = reinterpret_cast<double *>(base + off);
            off += round256(sizeof(double) * n);
            return d;
        };
        double *tmp = take(size_t(p.nn));
        double *Nt = take(4 * size_t(p.ntet));
        ApplyBufs bf;
        bf.xm = take(size_t(bem_ld(p.topo[0].nv)));
        bf.xs = take(size_t(bem_ld(p.topo[1].nv)));
        for (int w = 0; w < 2; ++w) {
            double *P = take(size_t(sym_partials_doubles(p.topo[w].nv)));
            bf.P[w] = p.surf[w].sym ? P : nullptr;
        }
        const int64_t n = p.n();
        coupled_apply_linear_bufs(p, phi, F, s, bf);
        fem_nonlinear_buf(p, scheme, phi, tmp, Nt, s);
        vec_axpby(p.nn, 1.0, tmp, 1.0, F, s);
        vec_axpby(n, -1.0, p.d_b, 1.0, F, s);
        PB_HIP(hipGetLastError());
        return PBFB_OK;
    } catch (const Error &e) {
        set_error(e.msg);
        return e.code;
    } catch (const std::exception &e) {
        set_error(e.what());
        return PBFB_EDEVICE;
    }
}
