// extern "C" entry points, quadrature rules, error state, timers, scratch.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "pbfb_internal.hpp"

namespace pbfb {

static thread_local std::string g_error;
void set_error(const std::string &msg) { g_error = msg; }

// ---------------------------------------------------------------------------
// quadrature rules
// ---------------------------------------------------------------------------
// Gauss rule with 3 nodes on [0,1] for the weight (1-x)^alpha, by the
// Golub-Welsch method: eigen-decomposition (cyclic Jacobi rotations) of the
// symmetric tridiagonal Jacobi matrix of the Jacobi polynomials P^(alpha,0),
// mapped from [-1,1] to [0,1].
static void golub_welsch3(double alpha, double x[3], double w[3])
{
    const double be = 0.0;
    double J[3][3] = {{0}};
    for (int k = 0; k < 3; ++k) {
        const double s = 2.0 * k + alpha + be;
        double a;
        if (k == 0) a = (be - alpha) / (alpha + be + 2.0);
        else a = (be * be - alpha * alpha) / (s * (s + 2.0));
        J[k][k] = 0.5 * (a + 1.0);
    }
    for (int k = 1; k < 3; ++k) {
        const double s = 2.0 * k + alpha + be;
        const double b2 = 4.0 * k * (k + alpha) * (k + be) * (k + alpha + be) / (s * s * (s + 1.0) * (s - 1.0));
        J[k][k - 1] = J[k - 1][k] = 0.5 * std::sqrt(b2);
    }
    double Q[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = std::fabs(J[0][1]) + std::fabs(J[0][2]) + std::fabs(J[1][2]);
        if (off < 1e-300) break;
        for (int pI = 0; pI < 2; ++pI)
            for (int qI = pI + 1; qI < 3; ++qI) {
                if (std::fabs(J[pI][qI]) < 1e-300) continue;
                const double th = 0.5 * std::atan2(2.0 * J[pI][qI], J[qI][qI] - J[pI][pI]);
                const double c = std::cos(th), sn = std::sin(th);
                for (int k = 0; k < 3; ++k) { // J <- J G
                    const double a = J[k][pI], b = J[k][qI];
                    J[k][pI] = c * a - sn * b;
                    J[k][qI] = sn * a + c * b;
                }
                for (int k = 0; k < 3; ++k) { // J <- G^T J
                    const double a = J[pI][k], b = J[qI][k];
                    J[pI][k] = c * a - sn * b;
                    J[qI][k] = sn * a + c * b;
                }
                for (int k = 0; k < 3; ++k) {
                    const double a = Q[k][pI], b = Q[k][qI];
                    Q[k][pI] = c * a - sn * b;
                    Q[k][qI] = sn * a + c * b;
                }
            }
    }
    const double mu0 = 1.0 / (alpha + 1.0); // int_0^1 (1-x)^alpha
    int ord[3] = {0, 1, 2};
    std::sort(ord, ord + 3, [&](int a, int b) { return J[a][a] < J[b][b]; });
    for (int i = 0; i < 3; ++i) {
        x[i] = J[ord[i]][ord[i]];
        w[i] = mu0 * Q[0][ord[i]] * Q[0][ord[i]];
    }
}

static Rules make_rules()
{
    Rules R;
    // symmetric 6-point degree-4 rule (Strang & Fix; Dunavant 1985), two S21 orbits
    const double a1 = 0.445948490915964886318329253883, w1 = 0.223381589678011465944640566;
    const double a2 = 0.091576213509770743459571463402, w2 = 0.109951743655321867388692766;
    const double orb[2][2] = {{a1, w1}, {a2, w2}};
    int q = 0;
    for (int o = 0; o < 2; ++o) {
        const double a = orb[o][0], b = 1.0 - 2.0 * a;
        const double pts[3][3] = {{b, a, a}, {a, b, a}, {a, a, b}};
        for (int k = 0; k < 3; ++k, ++q) {
            for (int d = 0; d < 3; ++d) R.tri_bary[q][d] = pts[k][d];
            R.tri_w[q] = orb[o][1];
        }
    }
    // conical product tet rule: x ~ (1-x)^2, y ~ (1-y), z ~ 1 (Stroud)
    double x2[3], w2j[3], x1[3], w1j[3], x0[3], w0j[3];
    golub_welsch3(2.0, x2, w2j);
    golub_welsch3(1.0, x1, w1j);
    golub_welsch3(0.0, x0, w0j);
    q = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            for (int k = 0; k < 3; ++k, ++q) {
                const double X = x2[i], Y = x1[j] * (1.0 - X), Z = x0[k] * (1.0 - X) * (1.0 - x1[j]);
                R.tet_bary[q][0] = 1.0 - X - Y - Z;
                R.tet_bary[q][1] = X;
                R.tet_bary[q][2] = Y;
                R.tet_bary[q][3] = Z;
                R.tet_w[q] = 6.0 * w2j[i] * w1j[j] * w0j[k];
            }
    // 4-point Gauss-Legendre on [0,1]
    const double g1 = 0.339981043584856264802665759103, g2 = 0.861136311594052575223946488893;
    const double v1 = 0.652145154862546142626936050778, v2 = 0.347854845137453857373063949222;
    const double gx[4] = {-g2, -g1, g1, g2}, gw[4] = {v2, v1, v1, v2};
    for (int i = 0; i < 4; ++i) {
        R.gl_x[i] = 0.5 * (gx[i] + 1.0);
        R.gl_w[i] = 0.5 * gw[i];
    }
    return R;
}

const Rules &rules()
{
    static const Rules R = make_rules();
    return R;
}

// ---------------------------------------------------------------------------
// memory
// ---------------------------------------------------------------------------
void Arena::release()
{
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
}

void *scratch_bytes(Problem &p, int slot, size_t bytes)
{
    ScratchBuf &b = p.scr[slot];
    if (b.bytes < bytes) {
        if (b.ptr) PB_HIP(hipFree(b.ptr));
        b.ptr = nullptr;
        b.bytes = 0;
        PB_HIP(hipMalloc(&b.ptr, bytes));
        b.bytes = bytes;
    }
    return b.ptr;
}

void release_scratch(Problem &p, int slot)
{
    ScratchBuf &b = p.scr[slot];
    if (b.ptr) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
}

void release_all_scratch(Problem &p)
{
    for (int i = 0; i < SCR_N; ++i) release_scratch(p, i);
}

void release_device_state(Problem &p)
{
    release_all_scratch(p);
    p.mesh_arena.release();
    for (int w = 0; w < NSURF; ++w) {
        p.bem_arena[w].release();
        p.surf[w].sides.clear();
        p.surf[w].tile = -1;
        p.bem_topo_ready[w] = false;
        p.bem_ready[w] = false;
    }
    p.topo_ready = p.geom_ready = p.val_ready = p.fm_ready = false;
    p.d_b = nullptr;
    p.d_q = nullptr;
}

double *Workspace::doubles(size_t n)
{
    const size_t want = sizeof(double) * (n ? n : 1);
    if (bytes < want) {
        if (ptr) PB_HIP(hipFree(ptr));
        ptr = nullptr;
        bytes = 0;
        held.store(0);
        PB_HIP(hipMalloc(&ptr, want));
        bytes = want;
        held.store(want);
    }
    return static_cast<double *>(ptr);
}

// ---------------------------------------------------------------------------
// event timers
// ---------------------------------------------------------------------------
void EventTimer::begin(int c, hipStream_t s)
{
    if (size_t(2 * used + 2) > ev.size()) {
        if (ev.size() < 8192) {
            size_t old = ev.size();
            ev.resize(std::max<size_t>(512, 2 * old));
            for (size_t i = old; i < ev.size(); ++i) PB_HIP(hipEventCreate(&ev[i]));
            cls.resize(ev.size() / 2);
            closed.resize(ev.size() / 2);
        } else {
            drain();
        }
    }
    cls[used] = c;
    closed[used] = 0;
    PB_HIP(hipEventRecord(ev[2 * used], s));
    open.push_back(used);
    ++used;
}

void EventTimer::end(hipStream_t s)
{
    const int i = open.back();
    open.pop_back();
    PB_HIP(hipEventRecord(ev[2 * i + 1], s));
    closed[i] = 1;
}

void EventTimer::drain()
{
    int keep = 0;
    for (int i = 0; i < used; ++i) {
        if (closed[i]) {
            float ms = 0.f;
            PB_HIP(hipEventSynchronize(ev[2 * i + 1]));
            PB_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
            sum_ms[cls[i]] += ms;
            cnt[cls[i]] += 1;
            continue;
        }
        // still open: move to the front, keeping its recorded start event
        if (keep != i) {
            std::swap(ev[2 * keep], ev[2 * i]);
            std::swap(ev[2 * keep + 1], ev[2 * i + 1]);
            cls[keep] = cls[i];
            closed[keep] = 0;
            for (int &o : open)
                if (o == i) o = keep;
        }
        ++keep;
    }
    used = keep;
}

void EventTimer::destroy()
{
    for (auto e : ev) (void)hipEventDestroy(e);
    ev.clear();
    cls.clear();
    closed.clear();
    open.clear();
    used = 0;
}

} // namespace pbfb

using namespace pbfb;

#define API_BEGIN try {
#define API_END                                                                                        \
    }                                                                                                  \
    catch (const pbfb::Error &e)                                                                       \
    {                                                                                                  \
        set_error(e.msg);                                                                              \
        return e.code;                                                                                 \
    }                                                                                                  \
    catch (const std::bad_alloc &)                                                                     \
    {                                                                                                  \
        set_error("host allocation failed");                                                           \
        return PBFB_ENOMEM;                                                                            \
    }                                                                                                  \
    catch (const std::exception &e)                                                                    \
    {                                                                                                  \
        set_error(e.what());                                                                           \
        return PBFB_EDEVICE;                                                                           \
    }                                                                                                  \
    return PBFB_OK;

// a problem whose context was destroyed is detached: only pbfb_problem_destroy accepts it
static Problem &live(pbfb_problem *pp)
{
    PB_CHECK(pp, PBFB_EINVAL, "null problem");
    PB_CHECK(pp->p.ctx, PBFB_ESTATE, "the problem's context was destroyed");
    return pp->p;
}
static const Problem &live(const pbfb_problem *pp) { return live(const_cast<pbfb_problem *>(pp)); }

static hipStream_t pick_stream(Problem &p, void *s)
{
    hipStream_t st = s ? static_cast<hipStream_t>(s) : p.ctx->stream;
    PB_HIP(hipSetDevice(p.ctx->device));
    p.last_stream = st;
    return st;
}

// row i (ascending vertex order) of the stored [K' | V'] of surface w, widened
// to FP64 and put back into the ascending column order (the device stores
// rows and columns in the Morton vertex order)
static void copy_bem_row(Problem &p, int w, int64_t i, double *K, double *V)
{
    const SurfaceTopo &T = p.topo[w];
    const int64_t nv = T.nv, ld = bem_ld(nv), k = T.minv[i];
    std::vector<double> row(ld);
    if (p.precision == PBFB_MIXED) {
        std::vector<float> rowf(ld);
        PB_HIP(hipMemcpy(rowf.data(), static_cast<const float *>(p.surf[w].B) + k * ld, sizeof(float) * ld,
                         hipMemcpyDeviceToHost));
        for (int64_t j = 0; j < ld; ++j) row[j] = rowf[j];
    } else {
        PB_HIP(hipMemcpy(row.data(), static_cast<const double *>(p.surf[w].B) + k * ld, sizeof(double) * ld,
                         hipMemcpyDeviceToHost));
    }
    for (int64_t j = 0; j < nv; ++j) {
        if (K) K[j] = row[T.minv[j]];
        if (V) V[j] = row[nv + T.minv[j]];
    }
}

// copy an FP64 vector argument to the device if it lives on the host
static const double *dev_in(Problem &p, int slot, const double *v, int64_t n, int mem, hipStream_t s)
{
    if (mem == PBFB_MEM_DEVICE) return v;
    double *d = scratch<double>(p, slot, n);
    PB_HIP(hipMemcpyAsync(d, v, sizeof(double) * n, hipMemcpyHostToDevice, s));
    return d;
}

extern "C" {

const char *pbfb_last_error(void) { return g_error.c_str(); }

pbfb_status pbfb_ctx_create(int device, pbfb_ctx **out)
{
    API_BEGIN
    PB_CHECK(out, PBFB_EINVAL, "out is NULL");
    int n = 0;
    PB_HIP(hipGetDeviceCount(&n));
    PB_CHECK(device >= 0 && device < n, PBFB_EINVAL, "no such device");
    PB_HIP(hipSetDevice(device));
    auto *c = new pbfb_ctx;
    c->c.device = device;
    hipError_t e = hipStreamCreateWithFlags(&c->c.stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        PB_HIP(e);
    }
    (void)rules();
    try {
        noalloc_init(device); // device address of the allocation-free residual's work array
    } catch (...) {
        (void)hipStreamDestroy(c->c.stream);
        delete c;
        throw;
    }
    *out = c;
    API_END
}

void pbfb_ctx_destroy(pbfb_ctx *ctx)
{
    if (!ctx) return;
    {
        // problems still alive are detached (they keep their own device memory)
        std::lock_guard<std::mutex> lk(ctx->c.live_mu);
        for (Problem *q : ctx->c.live) q->ctx = nullptr;
        ctx->c.live.clear();
    }
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    (void)hipStreamDestroy(ctx->c.stream);
    for (hipStream_t st : ctx->c.setup_stream)
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    for (Workspace &w : ctx->c.asm_ws)
        if (w.ptr) (void)hipFree(w.ptr);
    delete ctx;
}

pbfb_status pbfb_problem_create(pbfb_ctx *ctx, int precision, pbfb_problem **out)
{
    API_BEGIN
    PB_CHECK(ctx && out, PBFB_EINVAL, "null argument");
    PB_CHECK(precision == PBFB_FP64 || precision == PBFB_MIXED, PBFB_EINVAL, "unknown precision");
    auto *p = new pbfb_problem;
    p->p.ctx = &ctx->c;
    p->p.device = ctx->c.device;
    p->p.precision = precision;
    {
        std::lock_guard<std::mutex> lk(ctx->c.live_mu);
        ctx->c.live.insert(&p->p);
    }
    *out = p;
    API_END
}

void pbfb_problem_destroy(pbfb_problem *pp)
{
    if (!pp) return;
    Problem &p = pp->p;
    if (p.ctx) {
        std::lock_guard<std::mutex> lk(p.ctx->live_mu);
        p.ctx->live.erase(&p);
    }
    (void)hipSetDevice(p.device);
    (void)hipDeviceSynchronize();
    p.timer.destroy();
    release_all_scratch(p);
    p.mesh_arena.release();
    for (int w = 0; w < NSURF; ++w) p.bem_arena[w].release();
    delete pp;
}

static void invalidate_geometry(Problem &p)
{
    p.geom_ready = p.val_ready = p.fm_ready = false;
    for (int w = 0; w < NSURF; ++w) p.bem_ready[w] = false;
}

pbfb_status pbfb_set_mesh(pbfb_problem *pp, int64_t n_nodes, const double *nodes, int64_t n_tets,
                          const int32_t *tets, int64_t n_tri_m, const int32_t *tri_m, int64_t n_tri_s,
                          const int32_t *tri_s)
{
    API_BEGIN
    PB_CHECK(pp && nodes && tets && tri_m && tri_s, PBFB_EINVAL, "null argument");
    PB_CHECK(n_nodes >= 4 && n_tets >= 1 && n_tri_m >= 4 && n_tri_s >= 4, PBFB_EINVAL, "mesh too small");
    PB_CHECK(n_nodes < (int64_t(1) << 31) && 4 * n_tets < (int64_t(1) << 31), PBFB_EINVAL, "mesh too large");
    Problem &p = live(pp);
    PB_HIP(hipSetDevice(p.ctx->device));
    (void)hipDeviceSynchronize();
    invalidate_geometry(p);
    p.topo_ready = false;
    for (int w = 0; w < NSURF; ++w) p.bem_topo_ready[w] = false;
    p.have_mesh = false;
    p.rs_x.clear();
    p.topo[2] = SurfaceTopo();
    p.nn = n_nodes;
    p.ntet = n_tets;
    p.ntet_m = 0;
    p.x.assign(nodes, nodes + 3 * n_nodes);
    for (double v : p.x) PB_CHECK(std::isfinite(v), PBFB_EINVAL, "non-finite node coordinate");
    p.tet.assign(tets, tets + 4 * n_tets);
    for (int32_t v : p.tet) PB_CHECK(v >= 0 && v < n_nodes, PBFB_EINVAL, "tet references a node out of range");
    build_surface_topo(p, 0, n_tri_m, tri_m);
    build_surface_topo(p, 1, n_tri_s, tri_s);
    p.have_mesh = true;
    API_END
}

pbfb_status pbfb_set_charges(pbfb_problem *pp, int64_t n, const double *xyz, const double *z)
{
    API_BEGIN
    PB_CHECK(pp && n >= 0 && (n == 0 || (xyz && z)), PBFB_EINVAL, "bad charge arguments");
    Problem &p = live(pp);
    p.nq = n;
    p.q.resize(4 * n);
    for (int64_t k = 0; k < n; ++k) {
        for (int d = 0; d < 3; ++d) p.q[4 * k + d] = xyz[3 * k + d];
        p.q[4 * k + 3] = z[k];
        for (int d = 0; d < 4; ++d) PB_CHECK(std::isfinite(p.q[4 * k + d]), PBFB_EINVAL, "non-finite charge");
    }
    p.fm_ready = false;
    p.have_charges = true;
    API_END
}

pbfb_status pbfb_set_params(pbfb_problem *pp, double eps_in, double eps_out, double kappa, double temperature_K)
{
    API_BEGIN
    PB_CHECK(pp, PBFB_EINVAL, "null problem");
    PB_CHECK(eps_in > 0 && eps_out > 0, PBFB_EINVAL, "permittivities must be positive");
    PB_CHECK(kappa >= 0 && std::isfinite(kappa), PBFB_EINVAL, "kappa must be >= 0");
    PB_CHECK(temperature_K > 0, PBFB_EINVAL, "temperature must be positive");
    Problem &p = live(pp);
    const bool perm = p.eps_m != eps_in || p.eps_s != eps_out;
    const bool kap = p.kappa != kappa;
    p.eps_m = eps_in;
    p.eps_s = eps_out;
    p.kappa = kappa;
    p.temp = temperature_K;
    // SI 2019 exact constants, vacuum permittivity CODATA 2018
    const double e = 1.602176634e-19, eps0 = 8.8541878128e-12, kB = 1.380649e-23, NA = 6.02214076e23;
    p.lB = e * e / (4.0 * M_PI * eps0 * kB * temperature_K) * 1e10; // Angstrom
    p.kT = kB * temperature_K * NA / 4184.0;                         // kcal/mol
    if (perm) p.val_ready = false; // stiffness and coupling values carry eps (the boundary operators do not)
    if (kap) p.bem_ready[1] = false;
    p.fm_ready = false;
    p.have_params = true;
    API_END
}

pbfb_status pbfb_get_sizes(const pbfb_problem *pp, int64_t *n_nodes, int64_t *n_m, int64_t *n_s, int64_t *n_unknowns,
                           int64_t *hbm_bytes)
{
    API_BEGIN
    PB_CHECK(pp, PBFB_EINVAL, "null problem");
    const Problem &p = live(pp);
    PB_CHECK(p.have_mesh, PBFB_ESTATE, "no mesh");
    if (n_nodes) *n_nodes = p.nn;
    if (n_m) *n_m = p.topo[0].nv;
    if (n_s) *n_s = p.topo[1].nv;
    if (n_unknowns) *n_unknowns = p.n();
    if (hbm_bytes) {
        size_t b = p.mesh_arena.bytes;
        for (int w = 0; w < NSURF; ++w) b += p.bem_arena[w].bytes;
        for (int i = 0; i < SCR_N; ++i) b += p.scr[i].bytes;
        *hbm_bytes = int64_t(b);
    }
    API_END
}

pbfb_status pbfb_setup(pbfb_problem *pp, void *stream)
{
    API_BEGIN
    PB_CHECK(pp, PBFB_EINVAL, "null problem");
    Problem &p = live(pp);
    hipStream_t s = pick_stream(p, stream);
    ensure_all(p, s);
    PB_HIP(hipStreamSynchronize(s));
    API_END
}

pbfb_status pbfb_residual(pbfb_problem *pp, int scheme, const double *phi, double *F, int mem, void *stream)
{
    API_BEGIN
    PB_CHECK(pp && phi && F, PBFB_EINVAL, "null argument");
    PB_CHECK(scheme >= PBFB_LIN && scheme <= PBFB_T7, PBFB_EINVAL, "unknown scheme");
    Problem &p = live(pp);
    hipStream_t s = pick_stream(p, stream);
    ensure_all(p, s);
    const int64_t n = p.n();
    const double *dphi = dev_in(p, SCR_G3, phi, n, mem, s);
    double *dF = mem == PBFB_MEM_DEVICE ? F : scratch<double>(p, SCR_G4, n);
    double *tmp = scratch<double>(p, SCR_G5, n);
    coupled_apply_linear(p, dphi, dF, s);
    fem_nonlinear(p, scheme, dphi, tmp, s);
    vec_axpby(p.nn, 1.0, tmp, 1.0, dF, s);
    vec_axpby(n, -1.0, p.d_b, 1.0, dF, s);
    if (mem != PBFB_MEM_DEVICE) PB_HIP(hipMemcpyAsync(F, dF, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    PB_HIP(hipStreamSynchronize(s));
    API_END
}

pbfb_status pbfb_apply_jacobian(pbfb_problem *pp, int scheme, const double *phi, const double *v, double *Jv, int mem,
                                void *stream)
{
    API_BEGIN
    PB_CHECK(pp && phi && v && Jv, PBFB_EINVAL, "null argument");
    PB_CHECK(scheme >= PBFB_LIN && scheme <= PBFB_T7, PBFB_EINVAL, "unknown scheme");
    Problem &p = live(pp);
    hipStream_t s = pick_stream(p, stream);
    ensure_all(p, s);
    const int64_t n = p.n();
    const double *dphi = dev_in(p, SCR_G3, phi, n, mem, s);
    const double *dv = dev_in(p, SCR_G4, v, n, mem, s);
    double *dJ = mem == PBFB_MEM_DEVICE ? Jv : scratch<double>(p, SCR_G5, n);
    fem_assemble_jacobian(p, scheme, dphi, s);
    coupled_apply(p, dv, dJ, s);
    if (mem != PBFB_MEM_DEVICE) PB_HIP(hipMemcpyAsync(Jv, dJ, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    PB_HIP(hipStreamSynchronize(s));
    API_END
}

void pbfb_solve_opts_default(pbfb_solve_opts *o)
{
    if (!o) return;
    o->scheme_first = PBFB_T3;
    o->omega_auto = 1;
    o->omega_fixed = 1.0;
    o->tol_nl = 1e-3;
    o->tol_gr = 1e-6;
    o->tol_gr0 = 1e-3;
    o->tol_omega = 0.1;
    o->l_e = 0.35;
    o->omega0_first = 2.0;
    o->omega0_next = 1.0;
    o->omega_min = 0.0;
    o->omega_max = 4.0;
    o->max_newton = 50;
    o->max_omega_it = 50;
    o->gmres_restart = 200;
    o->max_gmres = 2000;
    o->krylov_fp32 = 0;
    o->precond = PBFB_PC_CHEB_SPAI;
    o->cheb_degree = 24;
    o->cheb_ratio = 200.0;
    o->hip_graph = 1;
    o->omega_method = PBFB_OMEGA_NEWTON;
    o->nonlinear_method = PBFB_NEWTON;
    o->r_e = 1.4;
    o->n_schedule = 0;
    for (int k = 0; k < 8; ++k) o->schedule[k] = PBFB_HS;
}

} // extern "C"

namespace pbfb {
void check_opts(const pbfb_solve_opts &O)
{
    PB_CHECK(O.gmres_restart >= 1 && O.gmres_restart <= 1000 && O.max_gmres >= 1, PBFB_EINVAL, "bad GMRES options");
    PB_CHECK(O.tol_gr > 0 && O.tol_gr0 > 0 && O.tol_nl >= 0, PBFB_EINVAL, "bad tolerances");
    PB_CHECK((O.precond == PBFB_PC_DIAG || O.precond == PBFB_PC_CHEB_SPAI) && O.cheb_degree >= 1 &&
                 O.cheb_degree <= 64 && O.cheb_ratio > 1.0,
             PBFB_EINVAL, "bad preconditioner options");
    PB_CHECK(O.omega_method >= PBFB_OMEGA_NEWTON && O.omega_method <= PBFB_OMEGA_BSEC_DF &&
                 O.omega_min <= O.omega_max && O.max_omega_it >= 1,
             PBFB_EINVAL, "bad relaxation-search options");
    PB_CHECK((O.nonlinear_method == PBFB_NEWTON || O.nonlinear_method == PBFB_PICARD) && O.r_e >= 0.0, PBFB_EINVAL,
             "bad nonlinear-iteration options");
    PB_CHECK(O.scheme_first == PBFB_T3 || O.scheme_first == PBFB_HS, PBFB_EINVAL, "bad scheme_first");
    PB_CHECK(O.n_schedule >= 0 && O.n_schedule <= 8, PBFB_EINVAL, "bad n_schedule");
    for (int k = 0; k < O.n_schedule; ++k)
        PB_CHECK(O.schedule[k] == PBFB_T3 || O.schedule[k] == PBFB_T5 || O.schedule[k] == PBFB_T7 ||
                     O.schedule[k] == PBFB_HS,
                 PBFB_EINVAL, "schedule entries must be PBFB_T3, PBFB_T5, PBFB_T7 or PBFB_HS");
}
} // namespace pbfb

extern "C" {

pbfb_status pbfb_solve(pbfb_problem *pp, const pbfb_solve_opts *o, pbfb_result *res, double *phi_out, int mem,
                       void *stream)
{
    API_BEGIN
    PB_CHECK(pp && res, PBFB_EINVAL, "null argument");
    pbfb_solve_opts def;
    pbfb_solve_opts_default(&def);
    const pbfb_solve_opts &O = o ? *o : def;
    check_opts(O);
    Problem &p = live(pp);
    hipStream_t s = pick_stream(p, stream);
    const int64_t n = p.n();
    double *dout = nullptr;
    if (phi_out) dout = mem == PBFB_MEM_DEVICE ? phi_out : scratch<double>(p, SCR_G12, 2 * n);
    pbfb_status st = solve(p, O, *res, dout, s);
    if (phi_out && mem != PBFB_MEM_DEVICE) {
        PB_HIP(hipMemcpyAsync(phi_out, dout, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, s));
        PB_HIP(hipStreamSynchronize(s));
    }
    // other failures keep the message of the step that failed
    if (st == PBFB_ENOTCONV) set_error("iteration limit reached");
    else if (st == PBFB_ENAN) set_error("non-finite residual");
    return st;
    API_END
}

pbfb_status pbfb_solve_batch(pbfb_ctx *ctx, int n, pbfb_problem *const *probs, const pbfb_solve_opts *o,
                             pbfb_result *res, void *stream)
{
    API_BEGIN
    PB_CHECK(ctx && n >= 0 && (n == 0 || (probs && res)), PBFB_EINVAL, "bad batch arguments");
    pbfb_solve_opts def;
    pbfb_solve_opts_default(&def);
    const pbfb_solve_opts &O = o ? *o : def;
    check_opts(O);
    PB_HIP(hipSetDevice(ctx->c.device));
    hipStream_t s = stream ? static_cast<hipStream_t>(stream) : ctx->c.stream;
    std::vector<NewtonRun> runs;
    runs.reserve(n);
    for (int q = 0; q < n; ++q) {
        PB_CHECK(probs[q] && probs[q]->p.ctx == &ctx->c, PBFB_EINVAL, "problem missing or from another context");
        for (int r = 0; r < q; ++r) PB_CHECK(probs[r] != probs[q], PBFB_EINVAL, "a problem appears twice in the batch");
        probs[q]->p.last_stream = s;
        runs.emplace_back(&probs[q]->p, O, &res[q], nullptr);
    }
    std::vector<NewtonRun *> ptrs;
    for (auto &r : runs) ptrs.push_back(&r);
    run_newton(ptrs, s);
    pbfb_status first = PBFB_OK;
    for (int q = 0; q < n; ++q)
        if (res[q].status != PBFB_OK && first == PBFB_OK) {
            first = res[q].status;
            set_error(runs[q].message.empty() ? "instance " + std::to_string(q) + " failed" : runs[q].message);
        }
    return first;
    API_END
}

pbfb_status pbfb_energy(pbfb_problem *pp, const double *phi_lin, const double *phi_nl, double out[4], int mem,
                        void *stream)
{
    API_BEGIN
    PB_CHECK(pp && phi_lin && out, PBFB_EINVAL, "null argument");
    Problem &p = live(pp);
    hipStream_t s = pick_stream(p, stream);
    ensure_rhs(p, s);
    const int64_t n = p.n();
    const double *dl = dev_in(p, SCR_G3, phi_lin, n, mem, s);
    const double *dn = phi_nl ? dev_in(p, SCR_G4, phi_nl, n, mem, s) : nullptr;
    energy(p, dl, dn, out, s);
    API_END
}

pbfb_status pbfb_export_bem(pbfb_problem *pp, int surf, double *V, double *K)
{
    API_BEGIN
    PB_CHECK(pp && (surf == 0 || surf == 1), PBFB_EINVAL, "bad argument");
    Problem &p = live(pp);
    PB_CHECK(!p.bem_mf, PBFB_ESTATE, "matrix-free mode stores no boundary operator");
    hipStream_t s = pick_stream(p, nullptr);
    ensure_bem(p, surf, s);
    const int64_t nv = p.topo[surf].nv;
    for (int64_t i = 0; i < nv; ++i)
        copy_bem_row(p, surf, i, K ? K + i * nv : nullptr, V ? V + i * nv : nullptr);
    API_END
}

pbfb_status pbfb_export_bem_rows(pbfb_problem *pp, int surf, int64_t n_rows, const int64_t *rows, double *V,
                                 double *K)
{
    API_BEGIN
    PB_CHECK(pp && (surf == 0 || surf == 1) && n_rows >= 0 && (rows || n_rows == 0), PBFB_EINVAL, "bad argument");
    Problem &p = live(pp);
    PB_CHECK(!p.bem_mf, PBFB_ESTATE, "matrix-free mode stores no boundary operator");
    const int64_t nv = p.topo[surf].nv;
    for (int64_t r = 0; r < n_rows; ++r) PB_CHECK(rows[r] >= 0 && rows[r] < nv, PBFB_EINVAL, "row out of range");
    hipStream_t s = pick_stream(p, nullptr);
    ensure_bem(p, surf, s);
    for (int64_t r = 0; r < n_rows; ++r) copy_bem_row(p, surf, rows[r], K ? K + r * nv : nullptr, V ? V + r * nv : nullptr);
    API_END
}

pbfb_status pbfb_export_rhs(pbfb_problem *pp, double *b)
{
    API_BEGIN
    PB_CHECK(pp && b, PBFB_EINVAL, "null argument");
    Problem &p = live(pp);
    hipStream_t s = pick_stream(p, nullptr);
    ensure_rhs(p, s);
    PB_HIP(hipMemcpyAsync(b, p.d_b, sizeof(double) * p.n(), hipMemcpyDeviceToHost, s));
    PB_HIP(hipStreamSynchronize(s));
    API_END
}

pbfb_status pbfb_reset_operators(pbfb_problem *pp)
{
    API_BEGIN
    PB_CHECK(pp, PBFB_EINVAL, "null problem");
    invalidate_geometry(pp->p);
    API_END
}

pbfb_status pbfb_set_bem_mode(pbfb_problem *pp, int mode)
{
    API_BEGIN
    PB_CHECK(pp && (mode == PBFB_BEM_DENSE || mode == PBFB_BEM_MATRIX_FREE), PBFB_EINVAL, "bad boundary-operator mode");
    Problem &p = live(pp);
    const bool mf = mode == PBFB_BEM_MATRIX_FREE;
    PB_CHECK(!(mf && p.two_field()), PBFB_EINVAL, "the two-field form needs dense boundary operators");
    if (mf != p.bem_mf) {
        p.bem_mf = mf;
        for (int w = 0; w < NSURF; ++w) p.bem_ready[w] = p.bem_topo_ready[w] = false;
    }
    API_END
}

pbfb_status pbfb_set_two_field(pbfb_problem *pp, int64_t n_tets_m)
{
    API_BEGIN
    PB_CHECK(pp, PBFB_EINVAL, "null problem");
    Problem &p = live(pp);
    PB_CHECK(p.have_mesh, PBFB_ESTATE, "set_mesh must precede set_two_field");
    PB_CHECK(n_tets_m >= 0 && n_tets_m < p.ntet, PBFB_EINVAL, "n_tets_m must be in [0, n_tets)");
    PB_CHECK(!(n_tets_m > 0 && p.bem_mf), PBFB_EINVAL, "the two-field form needs dense boundary operators");
    if (n_tets_m != p.ntet_m) {
        p.ntet_m = n_tets_m;
        p.val_ready = false; // permittivity per tet and the Gamma_m coupling
        p.fm_ready = false;  // the load
    }
    API_END
}

pbfb_status pbfb_set_reaction_surface(pbfb_problem *pp, int64_t n_verts, const double *verts, int64_t n_tri,
                                      const int32_t *tri)
{
    API_BEGIN
    PB_CHECK(pp, PBFB_EINVAL, "null problem");
    Problem &p = live(pp);
    PB_CHECK(p.have_mesh, PBFB_ESTATE, "set_mesh must precede set_reaction_surface");
    PB_CHECK(n_verts == 0 || (verts && tri && n_verts >= 4 && n_tri >= 4), PBFB_EINVAL, "bad surface arguments");
    PB_CHECK(n_verts < (int64_t(1) << 31) && 3 * n_tri < (int64_t(1) << 31), PBFB_EINVAL, "surface too large");
    PB_HIP(hipSetDevice(p.ctx->device));
    (void)hipDeviceSynchronize();
    SurfaceTopo T;
    std::vector<double> xs;
    if (n_verts > 0) {
        xs.assign(verts, verts + 3 * n_verts);
        for (double v : xs) PB_CHECK(std::isfinite(v), PBFB_EINVAL, "non-finite vertex coordinate");
        build_surface_topo_on(T, n_verts, xs.data(), n_tri, tri);
    }
    // the device topology and geometry are built again with the new surface
    invalidate_geometry(p);
    p.topo_ready = false;
    p.bem_topo_ready[2] = false;
    p.topo[2] = std::move(T);
    p.rs_x = std::move(xs);
    API_END
}

pbfb_status pbfb_set_tile_shape(pbfb_problem *pp, int ta, int tb)
{
    API_BEGIN
    PB_CHECK(pp, PBFB_EINVAL, "null problem");
    int k = -1;
    if (!(ta == 0 && tb == 0)) {
        k = tile_shape_index(ta, tb);
        PB_CHECK(k >= 0, PBFB_EINVAL, "tile shape is not one of 16x32, 8x32, 8x64, 16x16, 8x16 (or 0x0 for tuned)");
    }
    Problem &p = live(pp);
    if (k != p.tile_fixed) {
        p.tile_fixed = k;
        for (int w = 0; w < NSURF; ++w) p.bem_ready[w] = false;
    }
    API_END
}

pbfb_status pbfb_get_tile_shape(const pbfb_problem *pp, int surf, int *ta, int *tb)
{
    API_BEGIN
    PB_CHECK(pp && (surf == 0 || surf == 1), PBFB_EINVAL, "bad argument");
    const int k = pp->p.surf[surf].tile;
    if (ta) *ta = k >= 0 ? TILE_SHAPES[k].ta : 0;
    if (tb) *tb = k >= 0 ? TILE_SHAPES[k].tb : 0;
    API_END
}

pbfb_status pbfb_timing_enable(pbfb_problem *pp, int on)
{
    API_BEGIN
    PB_CHECK(pp, PBFB_EINVAL, "null problem");
    pp->p.timing = on != 0;
    API_END
}

pbfb_status pbfb_timing(pbfb_problem *pp, int which, double *avg_ms, int64_t *count, int reset)
{
    API_BEGIN
    PB_CHECK(pp && which >= 0 && which < T_NCLASS, PBFB_EINVAL, "bad argument");
    Problem &p = live(pp);
    PB_HIP(hipSetDevice(p.ctx->device));
    p.timer.drain();
    const int64_t c = p.timer.cnt[which];
    if (avg_ms) *avg_ms = c ? p.timer.sum_ms[which] / double(c) : 0.0;
    if (count) *count = c;
    if (reset)
        for (int i = 0; i < T_NCLASS; ++i) {
            p.timer.sum_ms[i] = 0.0;
            p.timer.cnt[i] = 0;
        }
    API_END
}

} // extern "C"
