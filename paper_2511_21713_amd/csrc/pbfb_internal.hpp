// Internal declarations of the pbfb library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <map>
#include <set>
#include <mutex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pbfb.h"

namespace pbfb {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);

struct Error {
    pbfb_status code;
    std::string msg;
};

#define PB_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            throw ::pbfb::Error{e_ == hipErrorOutOfMemory ? PBFB_ENOMEM : PBFB_EDEVICE,                \
                                std::string(#call) + ": " + hipGetErrorString(e_)};                   \
    } while (0)

#define PB_CHECK(cond, code, msg)                                                                      \
    do {                                                                                               \
        if (!(cond)) throw ::pbfb::Error{code, msg};                                                   \
    } while (0)

// ---------------------------------------------------------------------------
// quadrature rules (host copies; kernels receive them through constant memory)
// ---------------------------------------------------------------------------
struct Rules {
    double tri_bary[6][3], tri_w[6];   // symmetric degree-4 triangle rule, weights sum to 1
    double tet_bary[27][4], tet_w[27]; // conical product rule, degree 5, weights sum to 1
    double gl_x[4], gl_w[4];           // Gauss-Legendre on [0,1], Sauter-Schwab directions
};
const Rules &rules();
void upload_rules(hipStream_t s);

// ---------------------------------------------------------------------------
// device memory owned by a problem
// ---------------------------------------------------------------------------
struct Arena {
    std::vector<void *> ptrs;
    size_t bytes = 0;
    template <class T> T *alloc(size_t n) {
        void *p = nullptr;
        size_t b = sizeof(T) * (n ? n : 1);
        PB_HIP(hipMalloc(&p, b));
        ptrs.push_back(p);
        bytes += b;
        return static_cast<T *>(p);
    }
    template <class T> T *upload(const std::vector<T> &v, hipStream_t s) {
        T *d = alloc<T>(v.size());
        if (!v.empty()) PB_HIP(hipMemcpyAsync(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s));
        return d;
    }
    void release();
    ~Arena() { release(); }
};

// Tile shapes of the regular assembly: ta target x tb source Morton-ordered
// triangles per workgroup, one triangle pair per thread.  The shape of each
// (precision, kernel, size class) is chosen at run time by timing every
// candidate on a sample of the actual surface (tile_tune in kernels_bem.hip).
struct TileShape {
    int ta, tb;
};
constexpr TileShape TILE_SHAPES[] = {{16, 32}, {8, 32}, {8, 64}, {16, 16}, {8, 16}};
constexpr int N_TILE_SHAPES = int(sizeof(TILE_SHAPES) / sizeof(TILE_SHAPES[0]));
constexpr int MAXS = 24; // slots per local vertex in a block (max triangles of a block at one vertex)
int tile_shape_index(int ta, int tb); // -1 if not a candidate
constexpr int MAXRING = 64; // largest 1-ring (vertex and its neighbours) of the approximate inverse

// Blocks of `bs` consecutive Morton-ordered triangles (one side of a tile
// shape): nb blocks, S = sum of their vertex counts; per block its first
// local-vertex index and vertex count; per local vertex (block, k) its
// operator index (vid: the surface vertex's position in the Morton vertex
// order, the row / column of the stored operator; ascending within a block)
// and the MAXS (triangle-in-block * 3 + corner) slots touching it (-1
// padded); ms_max = the largest slot count of any vertex in any block.
// A greedy colouring of the blocks such that two blocks of one colour share
// no vertex: col_blk[col_ptr[c] .. col_ptr[c + 1]) lists the blocks of
// colour c, ascending.  Tiles whose target blocks share one colour and whose
// source blocks share one colour touch disjoint operator entries, so such a
// set of tiles can add into the operator in one launch without atomics.
struct BlockSide {
    int bs = 0, ms_max = 0;
    int64_t nb = 0, S = 0;
    std::vector<int32_t> pref, nvb, slots, vid;
    int ncolor = 0;
    std::vector<int32_t> col_ptr, col_blk;
};
struct BlockSideDev {
    int bs = 0;
    int64_t nb = 0, S = 0;
    int32_t *pref = nullptr, *nvb = nullptr, *slots = nullptr, *vid = nullptr;
    int32_t *col_blk = nullptr;
};

// host-side topology of one boundary surface
constexpr int NSURF = 3; // Gamma_m, Gamma_s, independent Gamma_m mesh (two-field form)

struct SurfaceTopo {
    int64_t nv = 0, nt = 0;
    std::vector<int32_t> g;            // local vertex -> FEM node (ascending)
    std::vector<int32_t> tri;          // 3*nt local vertex ids, original order
    std::vector<int32_t> v2t_ptr, v2t; // vertex -> (tri*3 + local index)
    std::vector<int32_t> morton;       // Morton position -> triangle id
    // Morton vertex order (first appearance along the Morton triangle order):
    // the row / column order of the stored dense operator.  mvert[k] = local
    // vertex at position k, minv = its inverse, gmv[k] = g[mvert[k]]
    std::vector<int32_t> mvert, minv, gmv;
    // regular-assembly blocks of each block size in use (over Morton-ordered
    // triangles), built on first use
    std::map<int, BlockSide> sides;
    // touching pairs (tau, sigma) sharing at least one vertex, grouped by tau
    std::vector<int32_t> tp_ptr, tp_sig;
    // 1-ring pattern of the sparse approximate inverse
    std::vector<int32_t> ring_ptr, ring;
    int max_ring = 0;
    // 3-ring pattern of the near-field single layer (matrix-free mode), built on first use
    std::vector<int32_t> nf_ptr, nf_col;
    // in the Morton vertex order: pairs k' > k within two rings (where
    // touching-pair blocks can make the stored V' unsymmetric)
    std::vector<int32_t> d2_ptr, d2_col;
};

struct SurfaceDev {
    int64_t nv = 0, nt = 0;
    int32_t *g = nullptr, *tri = nullptr, *v2t_ptr = nullptr, *v2t = nullptr;
    // vertex coordinates, indexed through g (the FEM nodes, or the own
    // vertices of an independent Gamma_m mesh)
    const double *x = nullptr;
    // independent Gamma_m mesh (two-field form): the tet holding each vertex
    // and its 4 barycentric coordinates there (the trace of u by P1
    // interpolation); null for a surface made of FEM nodes
    int32_t *itet = nullptr;
    double *iw = nullptr;
    int32_t *mvert = nullptr, *minv = nullptr, *gmv = nullptr; // Morton vertex order (SurfaceTopo)
    double *qp = nullptr, *nrm = nullptr, *area = nullptr; // original order: 18, 3, 1 per triangle
    // Morton-ordered triangle data for the regular assembly
    int32_t *m_tri = nullptr;
    double *m_qp = nullptr, *m_nrm = nullptr, *m_area = nullptr; // FP64 evaluation
    double *m_cen = nullptr;                                     // FP32 evaluation: FP64 centroids,
    float *m_qf = nullptr, *m_nf = nullptr;                      // FP32 offsets from them, FP32 normals
    std::map<int, BlockSideDev> sides; // device copies of the block tables in use (bem arena)
    int tile = -1;                      // tile shape of the last assembly (index into TILE_SHAPES)
    // matrix-free mode: touching-pair blocks kept resident (18 per pair: V then K),
    // Morton position of each triangle
    double *tpv = nullptr;
    int32_t *mpos = nullptr;
    int32_t *tp_ptr = nullptr, *tp_sig = nullptr, *tp_tau = nullptr, *morton = nullptr;
    int64_t ntp = 0;
    int32_t *cslot = nullptr; // FEM-row slot of the coupling entry per (v2t entry, b)
    // matrix-free mode: near-field V' on the 3-ring pattern (rows ascending)
    int32_t *nf_ptr = nullptr, *nf_col = nullptr, *nf_row = nullptr;
    double *nf_val = nullptr;
    int64_t nf_nnz = 0;
    // assembled dense operator in the Morton vertex order: row k (vertex
    // mvert[k]) = [K'_k (nv) | V'_k (nv)], columns in the same order, FP64 or FP32
    void *B = nullptr;
    double *vdiag = nullptr; // diagonal of the signed single-layer block V' (ascending vertex order)
    // symmetric storage use: the regular part of V' is bitwise symmetric, and
    // Delta_kl = V'_kl - V'_lk (l > k in the Morton order, two-ring pattern) carries the rest
    bool sym = false;
    int32_t *d_ptr = nullptr, *d_col = nullptr;
    double *d_val = nullptr;
    // sparse approximate inverse of V' on the 1-ring pattern (GMRES preconditioner)
    int32_t *ring_ptr = nullptr, *ring = nullptr;
    double *spai = nullptr;
};

// Device workspace shared by the problems of a context for their dense
// assembly (the mirrored double layer of a square-tile assembly, vertex
// coordinates, touching-pair blocks): grown on demand, never shrunk, freed
// with the context.  One assembly uses it at a time (the mutex is held until
// the assembly's stream has drained).
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
    std::atomic<size_t> held{0}; // bytes, readable without the mutex (admission by HBM footprint)
    std::mutex mu;
    double *doubles(size_t n);
};

struct Problem;
// assemblies of one context that may run at once (the device setup of a
// batch runs on this many host threads and streams)
constexpr int N_ASM_WS = 4;

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    Workspace asm_ws[N_ASM_WS];
    hipStream_t setup_stream[N_ASM_WS] = {}; // streams of a batch's parallel device setup, created on first use
    std::mutex setup_mu;                     // guards their creation
    // tuned tile shape per (precision, kernel, size class); tune_mu guards it
    // and serialises the tuning, so every problem of the context sees one choice
    std::mutex tune_mu;
    std::map<int, int> tile_choice;
    size_t ws_held() const
    {
        size_t b = 0;
        for (const Workspace &w : asm_ws) b += w.held.load();
        return b;
    }
    // problems created in this context and not yet destroyed
    std::mutex live_mu;
    std::set<Problem *> live;
};

enum TimerClass { T_APPLY = 0, T_GEMV = 1, T_SPMV = 2, T_ASM = 3, T_SING = 4, T_PREC = 5, T_NCLASS = 6 };

// HIP-event timing of launch ranges, accumulated per class.  Pairs may nest;
// when the event pool is full the closed pairs are folded into the sums and
// the open ones are kept.
struct EventTimer {
    std::vector<hipEvent_t> ev;   // pairs
    std::vector<int> cls;         // class of each recorded pair
    std::vector<char> closed;     // end recorded
    std::vector<int> open;        // stack of open pair indices
    int used = 0;
    double sum_ms[T_NCLASS] = {0};
    int64_t cnt[T_NCLASS] = {0};
    void begin(int c, hipStream_t s);
    void end(hipStream_t s);
    void drain();
    void destroy();
};

enum ScratchSlot {
    SCR_CHK, SCR_TRIF, SCR_Q, SCR_EPART, SCR_UR, SCR_B, SCR_DOT, SCR_XM, SCR_XS, SCR_TPTAU,
    SCR_G0, SCR_G1, SCR_G2, SCR_G3, SCR_G4, SCR_G5, SCR_G6, SCR_G7, SCR_G8, SCR_G9, SCR_G10, SCR_G11, SCR_G12,
    SCR_BASIS, SCR_BASIS32, SCR_HPART, SCR_HVEC, SCR_NRM, SCR_CNT, SCR_PZ, SCR_PT, SCR_PZB, SCR_PDK, SCR_LMAX, SCR_PCOEF, SCR_TETR, SCR_MF0, SCR_MF1, SCR_SYMP0, SCR_SYMP1,
    SCR_FM, SCR_PL, SCR_PN, SCR_CGX, SCR_CGV, SCR_PLOC, SCR_TSLOT, SCR_VOL, SCR_SYMP2, SCR_RLOC, SCR_OMEGA,
    SCR_N
};

struct ScratchBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct Problem {
    Ctx *ctx = nullptr; // null once the context is destroyed (detached problem)
    int device = 0;     // the context's device, kept for the problem's own release
    int precision = PBFB_FP64;
    bool have_mesh = false, have_charges = false, have_params = false;
    bool topo_ready = false, geom_ready = false, fm_ready = false, bem_ready[NSURF] = {false, false, false};
    bool val_ready = false; // FEM stiffness and coupling values (depend on the permittivities)
    bool bem_topo_ready[NSURF] = {false, false, false};
    int tile_fixed = -1; // tile shape forced by pbfb_set_tile_shape (index), -1: tuned
    bool bem_mf = false; // boundary operators applied matrix-free (no dense storage)
    // host copies
    int64_t nn = 0, ntet = 0, nq = 0;
    // two-field form (Sec. 2.3): the last ntet_m tets fill the solute (eps_m,
    // no reaction term), the load is the point charges, lambda_m is recovered
    // after the solve; 0: the shell-only form
    int64_t ntet_m = 0;
    int64_t ntet_i() const { return ntet - ntet_m; }
    bool two_field() const { return ntet_m > 0; }
    std::vector<double> x;
    std::vector<int32_t> tet;
    std::vector<double> q; // 4 per charge: x, y, z, valence
    // surfaces: Gamma_m, Gamma_s (both over FEM nodes) and, in the two-field
    // form, optionally an independent Gamma_m mesh (own vertices rs_x) that
    // carries lambda_m and the reaction potential (Sec. 2.3.1)
    SurfaceTopo topo[NSURF];
    std::vector<double> rs_x;
    bool has_rs() const { return topo[2].nv > 0; }
    int gm() const { return two_field() && has_rs() ? 2 : 0; } // the surface of lambda_m and u_r
    double eps_m = 0, eps_s = 0, kappa = 0, temp = 298.15, lB = 0, kT = 0;
    // device
    Arena mesh_arena, bem_arena[NSURF];
    ScratchBuf scr[SCR_N];
    double *d_x = nullptr, *d_tgeo = nullptr, *d_q = nullptr;
    int32_t *d_tet = nullptr, *d_n2t_ptr = nullptr, *d_n2t = nullptr, *d_slot4 = nullptr;
    // FEM rows in sliced ELL: slice q holds rows [64q, 64q + 64); its entry k
    // of row 64q + l sits at d_sptr[q] + 64 k + l for k below the slice width
    // (d_sptr[q + 1] - d_sptr[q]) / 64, in ascending column order; entries past
    // a row's length hold column = the row itself and value 0.
    int32_t *d_sptr = nullptr, *d_col = nullptr, *d_diag = nullptr;
    double *d_val0 = nullptr, *d_val = nullptr;
    float *d_val32 = nullptr;
    int64_t nnz = 0;     // stored entries (with the slice padding)
    int64_t nnz_row = 0; // nonzeros of the rows (without it)
    double *d_b = nullptr; // right-hand side, length n
    int *d_bad = nullptr;
    SurfaceDev surf[NSURF];
    int64_t n() const { return nn + topo[0].nv + topo[1].nv; }
    // timers
    bool timing = false;
    EventTimer timer;
    hipStream_t last_stream = nullptr;
};

// reusable device scratch buffers, grown on demand (hipFree synchronises)
void *scratch_bytes(Problem &p, int slot, size_t bytes);
template <class T> T *scratch(Problem &p, int slot, size_t n)
{
    return static_cast<T *>(scratch_bytes(p, slot, sizeof(T) * (n ? n : 1)));
}
void release_scratch(Problem &p, int slot);
void release_all_scratch(Problem &p);
// frees every device allocation of the problem (arenas and scratch) and marks
// all device state stale; the host copies (mesh, charges, parameters) stay,
// so the next call sets the problem up again
void release_device_state(Problem &p);

// host preprocessing (setup.hip)
void build_surface_topo(Problem &p, int which, int64_t ntri, const int32_t *tri);
// the same for triangles over vertices 0..nverts-1 at coordinates x
void build_surface_topo_on(SurfaceTopo &S, int64_t nverts, const double *x, int64_t ntri, const int32_t *tri);
const BlockSide &block_side(SurfaceTopo &S, int bs); // built on first use
constexpr int SLICE = 64; // FEM rows per sliced-ELL slice: one wavefront
// Krylov state of a batched GMRES instance (the state word every batched kernel reads)
// FIN: the cycle ended on the residual estimate; the step only adds the
// preconditioned update to x (no true-residual apply) and the solve is done
enum GSt { G_INIT = 0, G_ARN = 1, G_UPD = 2, G_RES = 3, G_DONE = 4, G_FAIL = 5, G_FIN = 6 };
void build_fem_topology(Problem &p, std::vector<int32_t> &sptr, std::vector<int32_t> &col,
                        std::vector<int32_t> &n2t_ptr, std::vector<int32_t> &n2t, std::vector<int32_t> &slot4,
                        std::vector<int32_t> &diag, std::vector<int32_t> cslot[2]);

// device setup and operators (kernels_*.hip, solver.hip)
void ensure_topology(Problem &p, hipStream_t s);
void ensure_geometry(Problem &p, hipStream_t s);
void ensure_values(Problem &p, hipStream_t s);
void ensure_rhs(Problem &p, hipStream_t s);
void ensure_bem(Problem &p, int surf, hipStream_t s);
void ensure_all(Problem &p, hipStream_t s);

// FEM element kernels (row gather over the tets around each node)
void fem_assemble_jacobian(Problem &p, int scheme, const double *u, hipStream_t s); // d_val = A + J(u)
void fem_assemble_linear(Problem &p, hipStream_t s);                                  // d_val = A
// matrix-free boundary rows of surface w: y = [K'|V'] x for the packed x =
// [u on the surface | lambda]; st (nullable): Krylov state word, the kernels
// return at once unless it is G_ARN or G_RES
void mf_apply(Problem &p, int w, const double *x, double *y, const int *st, hipStream_t s);
void mf_vdiag(Problem &p, int w, hipStream_t s); // diagonal of V' from the resident touching-pair blocks
// near-field V' on the 3-ring pattern and the 1-ring approximate inverse from it
void mf_spai(Problem &p, int w, hipStream_t s);
void near_pattern(SurfaceTopo &S); // host: the 3-ring pattern (nf_ptr, nf_col), once
void delta_pattern(SurfaceTopo &S); // host: the upper two-ring pattern (d2_ptr, d2_col), once
void fem_nonlinear(Problem &p, int scheme, const double *u, double *out, hipStream_t s);
// f_d terms of the relaxation search at the omega held in device memory
// (wdev); every kernel returns at once while *skip is nonzero
void fem_omega_terms_dev(Problem &p, int scheme, const double *u, const double *D, const double *wdev,
                         const int *skip, double *rN, double *rJ, double *rH, hipStream_t s);
double fem_energy_integral(Problem &p, const double *u_lin, const double *u_nl, hipStream_t s);

// coupled operator y = J x with the current CSR values (pack + GEMV + SpMV)
void coupled_apply(Problem &p, const double *x, double *y, hipStream_t s);
// work buffers of one apply: packed surface inputs (bem_ld(nv) each) and the
// FP64 column partials and V-item row sums of the symmetric use
// (sym_partials_doubles(nv) each, null where a surface is not stored
// symmetric)
struct ApplyBufs {
    double *xm = nullptr, *xs = nullptr;
    double *P[2] = {nullptr, nullptr};
};
int64_t sym_partials_doubles(int64_t nv);
void noalloc_init(int device); // noalloc.hip: once per device, with the device current
// A only (no J_N), with caller-provided buffers (no allocation, no timing)
void coupled_apply_linear_bufs(Problem &p, const double *x, double *y, hipStream_t s, const ApplyBufs &bufs);
// N_scheme(u) into out (FEM rows) with a caller-provided element buffer of 4 ntet doubles
void fem_nonlinear_buf(Problem &p, int scheme, const double *u, double *out, double *Nt, hipStream_t s);
void coupled_apply_linear(Problem &p, const double *x, double *y, hipStream_t s); // A only (no J_N)

// vector helpers
int64_t bem_ld(int64_t nv); // padded row length of the dense surface operator
void vec_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
void vec_mul(int64_t n, const double *a, const double *x, double *y, hipStream_t s);
void vec_add(int64_t n, const double *a, const double *b, double *y, hipStream_t s);
double dot(Problem &p, const double *a, const double *b, int64_t n, hipStream_t s);
void dots(Problem &p, int k, const double *const *a, const double *const *b, int64_t n, double *out, hipStream_t s);
// the same into device memory (out[0..k)), no host round trip; skip as above
void dots_dev(Problem &p, int k, const double *const *a, const double *const *b, int64_t n, double *out,
              const int *skip, hipStream_t s);

// energy
void energy(Problem &p, const double *phi_lin, const double *phi_nl, double out[4], hipStream_t s);
// two-field form: lam = V0^-1 ((1/2 M_m + K0_m) u|Gamma_m - [with_load] f_m) by
// conjugate gradients on the stored Gamma_m operator (V0 is symmetric positive
// definite); phi and lam are device vectors
void lambda_m_recover(Problem &p, const double *phi, bool with_load, double *lam, hipStream_t s);

// batched GMRES (gmres_batched.hip): one linear system per job, all advanced together
struct GmresJob {
    Problem *p;
    const double *b;
    double *x;
    const double *dinv;
    double tol;
    int restart, maxit;
    int iters, status;
    int basis32; // Krylov basis in FP32 (mixed precision only)
    int pc, cheb_k;       // preconditioner (PBFB_PC_*), Chebyshev terms
    double cheb_ratio;
    const double *lmax;   // device scalar: Gershgorin bound of diag(F)^-1 F
    int applies;          // out: operator applications that did work
    int graph;            // replay the Krylov step from a captured HIP graph
};
void batched_gmres(std::vector<GmresJob *> &jobs, hipStream_t s);
void build_precond(Problem &p, double *dinv, hipStream_t s);
void check_opts(const pbfb_solve_opts &o); // throws PBFB_EINVAL
void fem_gershgorin(Problem &p, double *lmax_dev, hipStream_t s); // bound of diag(F)^-1 F, F = A + J_N

// Newton driver (solver.hip): one state machine per instance
struct NewtonRun {
    Problem *p;
    pbfb_solve_opts o;
    pbfb_result *res;
    double *phi_out_dev;
    int phase = 0, k = 0, sch = PBFB_HS, status = 0;
    double tol = 0.0, omega_last = 1.0;
    double e_km1 = 0.0, e_km2 = 0.0; // e of the two previous nonlinear steps
    bool frozen = false;
    bool c_ready = false; // c already holds b - A Phi for the next step
    double *phil = nullptr, *phinl = nullptr, *phi = nullptr, *c = nullptr, *d = nullptr, *D = nullptr;
    double *pv = nullptr, *rv = nullptr, *rN = nullptr, *rJ = nullptr, *rH = nullptr, *dinv = nullptr;
    double *lmax = nullptr; // Chebyshev bound (device) and its partial maxima
    GmresJob job{};
    std::string message;
    std::chrono::steady_clock::time_point t0, t1;
    // relaxation search of the current step, run on the device (OmegaSearch
    // in device memory) for every searching instance of a batch together
    bool searching = false, searched = false;
    double omega = 1.0;
    void *om_dev = nullptr;  // the device state
    double om_host[4] = {0, 0, 0, 0}; // read back: done, omega, evaluations, fallback
    NewtonRun(Problem *p_, const pbfb_solve_opts &o_, pbfb_result *res_, double *out);
};
bool advance(NewtonRun &r, hipStream_t s);               // true: needs its linear solve
// advances every unfinished run to its next linear solve (its job appended to
// jobs) or to its end (appended to finished, if given); the relaxation
// searches of all runs between two linear solves run together on the device
void advance_all(std::vector<NewtonRun *> &runs, std::vector<GmresJob *> &jobs, std::vector<NewtonRun *> *finished,
                 hipStream_t s);
void run_newton(std::vector<NewtonRun *> &runs, hipStream_t s);
pbfb_status solve(Problem &p, const pbfb_solve_opts &o, pbfb_result &res, double *phi_out_dev, hipStream_t s);

} // namespace pbfb

struct pbfb_ctx {
    pbfb::Ctx c;
};
struct pbfb_problem {
    pbfb::Problem p;
};
