// Host driver and C ABI of libfld (see include/fld.h).
//
// The solve is device-driven: every CG iteration is a fixed sequence of
// kernels ("slot") that exit at once when the device flag `done` is set, so
// the host can queue (or replay as a hipGraph) a chunk of slots and only polls
// the flag between chunks.  Reliable updates (FP64 correction of E, true FP64
// residual, re-scaled inner residual) are decided on the device inside a slot.
#include <algorithm>
#include <chrono>
#include <functional>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fld.h"
#include "fld_band.hpp"
#include "fld_dense.hpp"

using namespace fld;

static_assert(sizeof(fld_solve_info) == sizeof(StepInfo) && offsetof(fld_solve_info, rel_resid) == offsetof(StepInfo, rel_resid) &&
                  offsetof(fld_solve_info, ms) == offsetof(StepInfo, ms),
              "device step record must match fld_solve_info");

namespace {

constexpr const char* kVersion = "fld-mi355x 0.2";
// longest segment of graph-replayed steps between two host reads (fld_steps)
constexpr int kStepSeg = 8;

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);                     \
            return FLD_EHIP;                                                                  \
        }                                                                                     \
    } while (0)

struct Level64 {
    int nx = 0, ny = 0;
    double *m = nullptr, *We = nullptr, *Wn = nullptr;  // row-major, unnormalised
};

// A level seen row-major (RM) or transposed (TR); line solves run along rows.
template <typename T>
struct View {
    int nx = 0, ny = 0;
    const T *m = nullptr, *We = nullptr, *Wn = nullptr;
};

template <typename T>
struct LevelT {
    int nx = 0, ny = 0;
    T *m = nullptr, *We = nullptr, *Wn = nullptr;     // row-major inner copy (/ mu)
    T *mT = nullptr, *WeT = nullptr, *WnT = nullptr;  // transposed copy (line smoother)
    T *bP = nullptr, *xP = nullptr;                   // vectors in the level's primary layout
    T *bQ = nullptr, *xQ = nullptr;                   // secondary layout (line); xQ = pre-smoothed x (point)
    T *xQ2 = nullptr, *xPT = nullptr;                 // band-fused sweeps: second Q buffer, P temporary
    bool tr = false;                                  // primary layout is the transposed one
    bool band = false;                                // band-fused sweeps on this level
    int Rp = 2, Rq = 2;                               // band heights in the P and Q layouts
    View<T> view(bool transposed) const {
        View<T> v;
        if (!transposed) { v.nx = nx; v.ny = ny; v.m = m; v.We = We; v.Wn = Wn; }
        else { v.nx = ny; v.ny = nx; v.m = mT; v.We = WeT; v.Wn = WnT; }
        return v;
    }
};

template <typename T>
struct Inner {
    std::vector<LevelT<T>> lv;
    T* Ainv = nullptr;
    double* Ywork = nullptr;  // coarse inverse set-up: forward solutions
    // a coarsest level above kCoarseMax cells: its inverse by block cyclic
    // reduction (FP64: staged coefficients, two levels' line blocks A, C and
    // C transposed, per eliminated line A^-1, E, F and their transposes, the whole
    // inverse Gw, which is Ainv itself in binary64) and the multi-workgroup
    // product
    bool dense = false;
    DenseGeom dg{};
    double *dd = nullptr, *aa = nullptr, *cc = nullptr;
    double *rA[2] = {nullptr, nullptr}, *rC[2] = {nullptr, nullptr}, *rCt[2] = {nullptr, nullptr};
    double *rAinv = nullptr, *rE = nullptr, *rF = nullptr, *rEt = nullptr, *rFt = nullptr, *Gw = nullptr;
    T *r = nullptr, *x = nullptr, *p[2] = {nullptr, nullptr}, *q = nullptr;
    int sub_first = -1;                   // first level of the one-workgroup coarse sub-cycle (-1: none)
    // Krylov-accelerated launched levels (mg_cycle KL_K / KL_W2): bit l of
    // kl_mask set for level l; c1 and A c1 of each (primary layout)
    unsigned kl_mask = 0;
    std::vector<T*> kc1, kv1;
    std::vector<T*> kb2;  // the second pass's b - s1 A c1 (band-fused levels)
    SubCycle<T> sub{};
    size_t sub_lds = 0;
    hipGraphExec_t chunk_exec = nullptr;  // captured chunk of CG iterations
    double* chunk_E = nullptr;            // solution pointer the chunk was captured for
    int chunk_len = 0;
};

}  // namespace

struct fld_ctx {
    int nx = 0, ny = 0, geom = 0;
    BCDev bc{};
    fld_options opt{};
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    // the coarsest inverse is built on a side stream, forked after the
    // hierarchy and joined by the first V-cycle that needs it
    hipStream_t setup_stream = nullptr;
    hipEvent_t setup_fork = nullptr, setup_join = nullptr;
    // the same fork and join inside stream captures (fld_steps) use events of
    // their own, so an event recorded into a graph is never recorded again
    // outside one
    hipEvent_t cap_fork = nullptr, cap_join = nullptr;
    bool setup_pending = false;
    std::string err;
    std::vector<void*> allocs;
    // metrics
    double *xf = nullptr, *yf = nullptr;
    Metrics met{};
    // assembled FP64 operator
    double *We = nullptr, *Wn = nullptr, *m = nullptr, *rhs = nullptr, *s = nullptr, *r64 = nullptr;
    double* mu = nullptr;  // device: max diagonal (inner normalisation)
    double* dt_lim = nullptr;  // device: coupling-limited sub-step length (fld_substep)
    // step-start copies: E^n of a sub-cycled step (its operator), or the (E, T)
    // a multi-step segment restarts from; per-step records of one segment
    double *Esave = nullptr, *Tsave = nullptr;
    fld_solve_info* seg_info = nullptr;
    int* seg_count = nullptr;
    const double *fx = nullptr, *fy = nullptr;  // caller's face mass fluxes (fld_set_mass_flux)
    double cv_Tref = 1.0, cv_p = 0.0;  // power-law heat capacity (fld_set_cv_law; p = 0: off)
    double* cvl = nullptr;             // its per-cell c_v at the assembled T^n
    double *bside = nullptr, *rside = nullptr;  // last assembly's per-side boundary terms (face fluxes)
    std::vector<Level64> h64;
    double* part = nullptr;
    double* part2 = nullptr;  // r.r partials of k_update (read while part holds p.q)
    double* part_rz = nullptr;  // r.z partials of the V-cycle's last sweep (summed by k_spmv)
    double* rz_sum = nullptr;   // their total, when summed apart (many partials); [1]: r_k+1 . z_k
    double* part_rzo = nullptr; // r_k+1 . z_k partials of k_update (flexible CG)
    bool flex = false;          // Polak-Ribiere beta (every cycle but the plain V-cycle)
    double* kpart = nullptr;    // partial sums of the Krylov-accelerated level
    KLScal* kscal = nullptr;    // its coefficients
    // line-sweep replay measurement (fld_profile_sweeps): while `sweeps_only`,
    // enqueue_vcycle queues only the line-sweep launches and counts them
    bool sweeps_only = false;
    int sweep_first = 0;        // replay only grid levels sweep_first .. sweep_first + sweep_levels - 1
    int sweep_levels = 0;       // (sweep_levels 0: to the last launched level)
    int sweep_launches = 0;
    double sweep_bytes = 0.0;
    Scalars* sc_sweep = nullptr;  // solver state of the replay (never done)
    int nrz = 0;                // their number (set when the V-cycle is queued)
    size_t npart = 0;
    Scalars* sc = nullptr;
    Scalars* hsc = nullptr;  // pinned mirror
    Scalars* hsc2 = nullptr;     // second pinned mirror (pipelined multi-step: two chunks in flight)
    hipEvent_t pev[2] = {nullptr, nullptr};  // their copies' completion
    // a captured multi-step graph (fld_steps_graph) has been replayed on this
    // context: host-driven solves on it are refused (see fld_solve)
    bool replayed = false;
    int last_iters = 0;          // CG iterations of the last host-driven solve (read-ahead prediction)
    int* err_flag = nullptr;
    int* herr = nullptr;     // pinned
    bool assembled = false;
    // inputs of the last assemble (for the gas update)
    const double *T = nullptr, *rho = nullptr, *kP = nullptr, *cv = nullptr;
    double dt = 0.0;
    Inner<float> i32;
    Inner<double> i64;
    // measurement of the line-sweep kernels: HIP events around every launch
    struct Prof {
        bool on = false;
        std::vector<hipEvent_t> ev;    // start/stop pairs, one per recorded launch
        std::vector<double> bytes;     // algorithmic bytes of that launch
        int* ran = nullptr;            // device flags: launch did work
        int* hran = nullptr;           // pinned copy
        int slots = 0, used = 0;       // capacity / slots used since the last harvest
        int64_t launches = 0;
        double ms = 0.0, total_bytes = 0.0;
    } prof;

    template <typename U>
    hipError_t alloc(U** p, size_t n) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, sizeof(U) * (n ? n : 1));
        if (e == hipSuccess) {
            allocs.push_back(q);
            *p = static_cast<U*>(q);
        }
        return e;
    }
};

namespace {

// Makes `st` wait for a coarsest-inverse set-up still running on the side
// stream (before the inverse is used, or its inputs rewritten).
inline fld_status join_setup(fld_ctx* ctx, hipStream_t st) {
    if (!ctx->setup_pending) return FLD_OK;
    HIPCHK(hipStreamWaitEvent(st, ctx->setup_join, 0));
    ctx->setup_pending = false;
    return FLD_OK;
}

}  // namespace

namespace {

inline dim3 tile_grid(int nx, int ny) { return dim3((nx + TBX - 1) / TBX, (ny + TRows - 1) / TRows); }
inline dim3 cell_grid(int nx, int ny) { return dim3((nx + TBX - 1) / TBX, (ny + TBY - 1) / TBY); }
inline dim3 blk2d() { return dim3(TBX, TBY); }
inline int grid1d(size_t n) {
    size_t b = (n + 255) / 256;
    return (int)(b < (size_t)k1DBlocksMax ? (b ? b : 1) : (size_t)k1DBlocksMax);
}
// k_update's grid: few enough r.r partials for every k_resid64 workgroup to
// sum them itself
inline int update_grid(size_t n) { return std::min(grid1d(n), 512); }

bool inner_is_float(const fld_ctx* c) { return c->opt.precision != FLD_FP64; }

template <typename T>
Inner<T>& inner(fld_ctx* c);
template <>
Inner<float>& inner<float>(fld_ctx* c) { return c->i32; }
template <>
Inner<double>& inner<double>(fld_ctx* c) { return c->i64; }

fld_status validate_options(const fld_options* o, std::string& err) {
    if (o->precision < 0 || o->precision > 2) { err = "precision"; return FLD_EINVAL; }
    if (o->limiter < 0 || o->limiter > 2) { err = "limiter"; return FLD_EINVAL; }
    if (o->norm < 0 || o->norm > 1) { err = "norm"; return FLD_EINVAL; }
    if (!(o->rel_tol > 0.0) || !(o->rel_tol < 1.0)) { err = "rel_tol must be in (0, 1)"; return FLD_EINVAL; }
    if (o->max_outer < 1 || o->max_inner < 1) { err = "max_outer / max_inner must be >= 1"; return FLD_EINVAL; }
    if (!(o->inner_rtol > 0.0) || !(o->inner_rtol < 1.0)) { err = "inner_rtol must be in (0, 1)"; return FLD_EINVAL; }
    if (o->mg_coarse_max < 1 || o->mg_coarse_max > kDenseMax) { err = "mg_coarse_max must be in [1, 4096]"; return FLD_EINVAL; }
    if (o->mg_coarse_op < 0 || o->mg_coarse_op > 1) { err = "mg_coarse_op"; return FLD_EINVAL; }
    if (o->smoother < 0 || o->smoother > 2) { err = "smoother"; return FLD_EINVAL; }
    if (o->chunk < 2 || (o->chunk & 1)) { err = "chunk must be even and >= 2"; return FLD_EINVAL; }
    if (o->mg_cycle < 0 || o->mg_cycle > 4) { err = "mg_cycle"; return FLD_EINVAL; }
    return FLD_OK;
}

// ---------------------------------------------------------------------------
// V-cycle and CG slot (queued on stream `st`)
// ---------------------------------------------------------------------------

// Coupling-limited sub-step length (Section 3.2.1, global sub-step rule):
// per-workgroup minimum over the cells of dbar T C_V / |G0| with
// G0 = kappa_P rho c (a_R T^4 - E) and C_V = rho c_v; a cell in exact
// equilibrium (G0 = 0) does not limit.
__global__ __launch_bounds__(256) void k_coupling_dt(int n, const double* __restrict__ E, const double* __restrict__ T,
                                                     const double* __restrict__ rho, const double* __restrict__ kP,
                                                     const double* __restrict__ cv, double dbar, double* part) {
    __shared__ double sh[16];
    double v = INFINITY;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const double t = T[c], t2 = t * t;
        const double g = kP[c] * rho[c] * kC * (kARad * (t2 * t2) - E[c]);
        if (g != 0.0) v = fmin(v, dbar * t * (rho[c] * cv[c]) / fabs(g));
    }
    const double m = block_min(v, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// Heat capacity of the power-law stand-in for a nonlinear equation of state,
// re-evaluated from T before every step's assembly (Section 3.2.1, the C_V
// step of the radiation-subsystem algorithm): c_v = c_v,ref (T / T_ref)^p.
__global__ __launch_bounds__(256) void k_cv_law(int n, const double* __restrict__ cv_ref,
                                                const double* __restrict__ T, double inv_Tref, double p,
                                                double* __restrict__ out) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
        out[c] = cv_ref[c] * pow(T[c] * inv_Tref, p);
}

// Minimum of nb partials into *out (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void k_reduce_min(const double* part, int nb, double* out) {
    __shared__ double sh[16];
    double v = INFINITY;
    for (int b = threadIdx.x; b < nb; b += 1024) v = fmin(v, part[b]);
    const double m = block_min(v, sh);
    if (threadIdx.x == 0) *out = m;
}

// Radiative flux through every face from the last assembly (Section 3.2.1
// flux formula), positive along +x / +y: interior faces W (E_lo - E_hi) /
// (dt dS), boundary faces the outward flux of their side's row terms,
// (d E_1 - r) / (dt dS), negated on the lower sides; faces of zero area carry
// none.  Writes w F, or adds it with acc.
__global__ __launch_bounds__(256) void k_face_flux(Metrics g, const double* __restrict__ We,
                                                   const double* __restrict__ Wn, const double* __restrict__ bside,
                                                   const double* __restrict__ rside, const double* __restrict__ E,
                                                   double dt, double w, int acc, double* Fx, double* Fy) {
    const int nx = g.nx, ny = g.ny;
    const int nfx = (nx + 1) * ny, nfy = nx * (ny + 1);
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nfx + nfy; f += gridDim.x * blockDim.x) {
        double F = 0.0;
        if (f < nfx) {
            if (!Fx) continue;
            const int j = f / (nx + 1), i = f - j * (nx + 1);
            const double dS = g.sx[i] * g.vy[j];
            if (dS > 0.0) {
                const size_t c = (size_t)j * nx + i;
                if (i > 0 && i < nx) F = We[c - 1] * (E[c - 1] - E[c]) / (dt * dS);
                else if (i == 0) F = -(bside[j] * E[c] - rside[j]) / (dt * dS);
                else F = (bside[ny + j] * E[c - 1] - rside[ny + j]) / (dt * dS);
            }
            Fx[f] = acc ? Fx[f] + w * F : w * F;
        } else {
            if (!Fy) continue;
            const int q = f - nfx, j = q / nx, i = q - j * nx;
            const double dS = g.ax[i] * g.sy[j];
            if (dS > 0.0) {
                const size_t c = (size_t)j * nx + i;
                if (j > 0 && j < ny) F = Wn[c - nx] * (E[c - nx] - E[c]) / (dt * dS);
                else if (j == 0) F = -(bside[2 * ny + i] * E[c] - rside[2 * ny + i]) / (dt * dS);
                else F = (bside[2 * ny + nx + i] * E[c - nx] - rside[2 * ny + nx + i]) / (dt * dS);
            }
            Fy[q] = acc ? Fy[q] + w * F : w * F;
        }
    }
}

inline bool is_line(const fld_options& o) { return o.smoother == FLD_SMOOTH_LINE || o.smoother == FLD_SMOOTH_LINE_SPLIT; }

// Chunking of a row of n cells for k_line: K chunks (power of two, <= 512) of
// L cells (2 <= L <= 8).
inline void line_params(int n, int& K, int& L) {
    int want = (n + kLineMaxL - 1) / kLineMaxL;
    K = 1;
    while (K < want && K < kLineWG) K <<= 1;
    L = (n + K - 1) / K;
    if (L < 2) L = 2;
}

template <typename T, int MODE, int DOT>
int launch_line(fld_ctx* c, const View<T>& v, int par, const T* b, T* x, const T* ec, int nxc, int nb_prev,
                hipStream_t st) {
    const int nl = (v.ny - par + 1) / 2;
    if (nl <= 0) return 0;
    int K, L;
    line_params(v.nx, K, L);
    const int lpw = kLineWG / K;
    const int grid = (nl + lpw - 1) / lpw;
    auto& P = c->prof;
    int slot = -1;
    // algorithmic bytes: solved rows read m, W_e, b and write x; W_n of every
    // row; x of the neighbour rows unless zero; the coarse correction (1/4)
    const double n = (double)v.nx * v.ny, half = (double)nl * v.nx;
    double words = 4.0 * half + n;
    if (MODE != LINE_ZERO) words += n - half;
    if (MODE == LINE_PROLONG) words += 0.25 * n;
    if (c->sweeps_only) {
        ++c->sweep_launches;
        c->sweep_bytes += words * sizeof(T);
    }
    if (P.on && P.used < P.slots) {
        slot = P.used++;
        P.bytes[slot] = words * sizeof(T);
        (void)hipEventRecord(P.ev[2 * slot], st);
    }
    if (L == kLineMaxL && K * kLineMaxL == v.nx)
        k_line<T, MODE, DOT, true><<<grid, kLineWG, 0, st>>>(v.nx, v.ny, K, L, par, v.m, v.We, v.Wn, b, x, ec, nxc,
                                                              T(1), DOT ? c->part_rz : c->part, nb_prev, c->sc,
                                                              slot >= 0 ? P.ran + slot : nullptr);
    else
        k_line<T, MODE, DOT, false><<<grid, kLineWG, 0, st>>>(v.nx, v.ny, K, L, par, v.m, v.We, v.Wn, b, x, ec, nxc,
                                                               T(1), DOT ? c->part_rz : c->part, nb_prev, c->sc,
                                                               slot >= 0 ? P.ran + slot : nullptr);
    if (slot >= 0) (void)hipEventRecord(P.ev[2 * slot + 1], st);
    return grid;
}

// Both half-sweeps of the rows of view v in one launch (k_band); returns the
// grid size (the number of r.z partials when DOT).
template <typename T, int MODE, int FIRST, bool OUT_T, bool WRITE_BT, bool DOT>
int launch_band(fld_ctx* c, const View<T>& v, int R, const T* b, const T* xin, const T* ec, int nxc, T* xout,
                T* bout, hipStream_t st, BandKL<T> kl = BandKL<T>{}) {
    int K, L;
    line_params(v.nx, K, L);
    const int grid = (v.ny + R - 1) / R;
    auto& P = c->prof;
    int slot = -1;
    // algorithmic bytes: m, W_e, W_n, b of every row and x written once; the
    // old x of the rows solved second (read by the rows solved first) unless
    // zero; the coarse correction; b written transposed
    const double n = (double)v.nx * v.ny;
    double words = 5.0 * n;
    if (MODE != LINE_ZERO) words += 0.5 * n;
    if (MODE == LINE_PROLONG) words += 0.25 * n;
    if (WRITE_BT) words += n;
    // a folded Krylov update: A c1 read and b - s1 A c1 stored (zero-start
    // sweep), or the level below's c1 read with its correction
    if (kl.v) words += MODE == LINE_ZERO ? 2.0 * n : MODE == LINE_PROLONG ? 0.25 * n : 0.0;
    if (c->sweeps_only) {
        ++c->sweep_launches;
        c->sweep_bytes += words * sizeof(T);
    }
    if (P.on && P.used < P.slots) {
        slot = P.used++;
        P.bytes[slot] = words * sizeof(T);
        (void)hipEventRecord(P.ev[2 * slot], st);
    }
    const size_t lds = band_lds_bytes<T>(v.nx, R, WRITE_BT);
    int* ran = slot >= 0 ? P.ran + slot : nullptr;
    k_band<T, kLineMaxL, MODE, FIRST, OUT_T, WRITE_BT, DOT><<<grid, kBandWG, lds, st>>>(
        v.nx, v.ny, R, K, L, v.m, v.We, v.Wn, b, xin, ec, nxc, xout, bout, DOT ? c->part_rz : c->part, c->sc, ran, kl);
    if (slot >= 0) (void)hipEventRecord(P.ev[2 * slot + 1], st);
    return grid;
}

// Adds the timed launches that did work to the totals (stream synchronised).
fld_status prof_harvest(fld_ctx* ctx) {
    auto& P = ctx->prof;
    if (!P.on || P.used == 0) return FLD_OK;
    HIPCHK(hipMemcpy(P.hran, P.ran, sizeof(int) * P.used, hipMemcpyDeviceToHost));
    for (int k = 0; k < P.used; ++k) {
        if (!P.hran[k]) continue;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, P.ev[2 * k], P.ev[2 * k + 1]));
        P.ms += ms;
        P.total_bytes += P.bytes[k];
        P.launches += 1;
    }
    HIPCHK(hipMemset(P.ran, 0, sizeof(int) * P.used));
    P.used = 0;
    return FLD_OK;
}

template <typename T>
void launch_transpose(int nx, int ny, const T* s0, const T* s1, T* d0, T* d1, const Scalars* sc, hipStream_t st) {
    dim3 g((nx + kTT - 1) / kTT, (ny + kTT - 1) / kTT), blk(kTT, 8);
    if (s1)
        k_transpose<T, 2><<<g, blk, 0, st>>>(nx, ny, s0, s1, nullptr, d0, d1, nullptr, sc);
    else
        k_transpose<T, 1><<<g, blk, 0, st>>>(nx, ny, s0, nullptr, nullptr, d0, nullptr, nullptr, sc);
}

// x = A^-1 b on the coarsest level (below a launched level): one workgroup
// up to kCoarseMax cells, the multi-workgroup product above.
template <typename T>
void coarse_solve(fld_ctx* c, Inner<T>& in, hipStream_t st) {
    LevelT<T>& cl = in.lv.back();
    const int n = cl.nx * cl.ny;
    if (in.dense)
        k_dense_solve<T, false><<<(n + kDenseRows - 1) / kDenseRows, kDenseThreads, 0, st>>>(in.dg, in.Ainv, cl.bP,
                                                                                            cl.xP, nullptr, c->sc);
    else
        k_coarse_solve<T, false><<<1, kCoarseSolveThreads, 0, st>>>(n, in.Ainv, cl.bP, cl.xP, nullptr, c->sc);
}

template <typename T>
void enqueue_vcycle_line(fld_ctx* c, Inner<T>& in, hipStream_t st) {
    const int L = (int)in.lv.size();
    const int Ld = in.sub_first > 0 ? in.sub_first : L - 1;  // grid levels smoothed with launches
    const bool fused = c->opt.smoother == FLD_SMOOTH_LINE;
    std::vector<T*> xpre(Ld);  // pre-smoothed x of each level (secondary layout)
    // the replay measurement can be limited to the finest levels
    auto skip = [&](int l) {
        return c->sweeps_only &&
               (l < c->sweep_first || (c->sweep_levels > 0 && l >= c->sweep_first + c->sweep_levels));
    };
    // pre-smoothing of level l and its residual restricted to level l + 1
    // kb: a Krylov level's second pass on a band-fused level folds
    // b <- b - s1 A c1 into its first sweep (the result also in kb.bout2)
    auto down = [&](int l, BandKL<T> kb = BandKL<T>{}) {
        if (skip(l)) return;
        LevelT<T>& a = in.lv[l];
        LevelT<T>& nxt = in.lv[l + 1];
        const View<T> vp = a.view(a.tr), vq = a.view(!a.tr);
        if (fused && a.band) {
            // rows of P (even, odd) -> x and b transposed into Q; rows of Q (even, odd)
            launch_band<T, LINE_ZERO, 0, true, true, false>(c, vp, a.Rp, a.bP, nullptr, nullptr, 0, a.xQ, a.bQ, st,
                                                            kb);
            launch_band<T, LINE_NORMAL, 0, false, false, false>(c, vq, a.Rq, a.bQ, a.xQ, nullptr, 0, a.xQ2, nullptr,
                                                                st);
            xpre[l] = a.xQ2;
        } else {
            launch_line<T, LINE_ZERO, 0>(c, vp, 0, a.bP, a.xP, nullptr, 0, 0, st);
            launch_line<T, LINE_NORMAL, 0>(c, vp, 1, a.bP, a.xP, nullptr, 0, 0, st);
            if (!c->sweeps_only) launch_transpose<T>(vp.nx, vp.ny, a.xP, a.bP, a.xQ, a.bQ, c->sc, st);
            launch_line<T, LINE_NORMAL, 0>(c, vq, 0, a.bQ, a.xQ, nullptr, 0, 0, st);
            launch_line<T, LINE_NORMAL, 0>(c, vq, 1, a.bQ, a.xQ, nullptr, 0, 0, st);
            xpre[l] = a.xQ;
        }
        const View<T> cv = nxt.view(nxt.tr);
        if (!c->sweeps_only)
            k_resid_restrict<T><<<tile_grid(vq.nx, vq.ny), blk2d(), 0, st>>>(vq.nx, vq.ny, vq.m, vq.We, vq.Wn, a.bQ,
                                                                          xpre[l], nxt.bP, cv.nx, cv.ny, c->sc);
    };
    auto coarse = [&]() {
        if (c->sweeps_only) {
            // line sweeps only (replay measurement)
        } else if ((void)join_setup(c, st), in.sub_first > 0) {
            LevelT<T>& f = in.lv[in.sub_first];
            k_subcycle<T><<<1, kSubThreads<T>, in.sub_lds, st>>>(in.sub, f.bP, f.xP, c->sc);
        } else {
            coarse_solve<T>(c, in, st);
        }
    };
    // prolongation of the correction from level l + 1 and post-smoothing of level l
    // bp: the level's right-hand side in P if not a.bP (a Krylov level's
    // second pass); ke: the level below is a Krylov level whose two-step
    // combination is folded into the prolongation
    auto up = [&](int l, const T* bp = nullptr, BandKL<T> ke = BandKL<T>{}) {
        if (skip(l)) return;
        LevelT<T>& a = in.lv[l];
        LevelT<T>& nxt = in.lv[l + 1];
        const View<T> vp = a.view(a.tr), vq = a.view(!a.tr);
        const View<T> cv = nxt.view(nxt.tr);
        const T* bP = bp ? bp : a.bP;
        if (fused && a.band) {
            // rows of Q (odd with the coarse correction, even) -> x transposed
            // into P; rows of P (odd, even), the last with r.z on the fine level
            launch_band<T, LINE_PROLONG, 1, true, false, false>(c, vq, a.Rq, a.bQ, xpre[l], nxt.xP, cv.nx, a.xPT,
                                                                nullptr, st, ke);
            if (l == 0) {
                c->nrz = launch_band<T, LINE_NORMAL, 1, false, false, true>(c, vp, a.Rp, bP, a.xPT, nullptr, 0,
                                                                            a.xP, nullptr, st);
            } else {
                launch_band<T, LINE_NORMAL, 1, false, false, false>(c, vp, a.Rp, bP, a.xPT, nullptr, 0, a.xP,
                                                                    nullptr, st);
            }
            return;
        }
        launch_line<T, LINE_PROLONG, 0>(c, vq, 1, a.bQ, a.xQ, nxt.xP, cv.nx, 0, st);
        launch_line<T, LINE_NORMAL, 0>(c, vq, 0, a.bQ, a.xQ, nullptr, 0, 0, st);
        if (!c->sweeps_only) launch_transpose<T>(vq.nx, vq.ny, a.xQ, nullptr, a.xP, nullptr, c->sc, st);
        if (l == 0) {
            // the last two sweeps of level 0 also accumulate r.z for CG
            const int nb1 = launch_line<T, LINE_NORMAL, 1>(c, vp, 1, a.bP, a.xP, nullptr, 0, 0, st);
            const int nb2 = launch_line<T, LINE_NORMAL, 1>(c, vp, 0, a.bP, a.xP, nullptr, 0, nb1, st);
            c->nrz = nb1 + nb2;
        } else {
            launch_line<T, LINE_NORMAL, 0>(c, vp, 1, a.bP, a.xP, nullptr, 0, 0, st);
            launch_line<T, LINE_NORMAL, 0>(c, vp, 0, a.bP, a.xP, nullptr, 0, 0, st);
        }
    };
    // the cycle from level l down; a Krylov-accelerated level K takes two
    // flexible-CG steps on A_K e = r_K, each preconditioned by the cycle from
    // K down (its coefficients and partial sums in slot K of kscal / kpart)
    // pend[l]: the Krylov level l + 1's combination x <- f1 c1 + f2 x, folded
    // into up(l)'s prolongation (band-fused level l)
    std::vector<BandKL<T>> pend(L);
    auto take = [&](int l) {
        BandKL<T> k = pend[l];
        pend[l] = BandKL<T>{};
        return k;
    };
    std::function<void(int)> cycle = [&](int l) {
        if (l == Ld) {
            coarse();
            return;
        }
        const bool krylov = l > 0 && ((in.kl_mask >> l) & 1u) && !c->sweeps_only;
        if (!krylov) {
            down(l);
            cycle(l + 1);
            up(l, nullptr, take(l));
            return;
        }
        LevelT<T>& a1 = in.lv[l];
        const View<T> v1 = a1.view(a1.tr);
        const int n1 = v1.nx * v1.ny;
        const int G = std::max(1, std::min((n1 + kKLThreads - 1) / kKLThreads, kKLMaxWG));
        const int single = sizeof(T) == 4 ? 1 : 0;
        double* part = c->kpart + (size_t)l * 3 * kKLMaxWG;
        KLScal* ks = c->kscal + l;
        // few partials: their consumers sum them (no separate reduction
        // launch); band-fused levels take the vector updates into their sweeps
        const bool fold = G <= kKLFoldMax;
        const bool band = fused && a1.band;
        const bool parent_band = fused && in.lv[l - 1].band;
        down(l);
        cycle(l + 1);
        up(l, nullptr, take(l));
        k_kl_dots<T, 0><<<G, kKLThreads, 0, st>>>(v1.nx, v1.ny, v1.m, v1.We, v1.Wn, a1.xP, a1.bP, in.kc1[l],
                                                  in.kv1[l], part, c->sc);
        BandKL<T> kb{};
        if (band) {
            if (!fold) k_kl_reduce<0><<<1, kRedThreads, 0, st>>>(part, G, ks, c->sc, single);
            kb.v = in.kv1[l];
            kb.part = fold ? part : nullptr;
            kb.G = G;
            kb.ks = ks;
            kb.bout2 = in.kb2[l];
        } else if (fold) {
            k_kl_axpy<T, true><<<G, kKLThreads, 0, st>>>(n1, a1.bP, in.kv1[l], part, G, ks, c->sc);
        } else {
            k_kl_reduce<0><<<1, kRedThreads, 0, st>>>(part, G, ks, c->sc, single);
            k_kl_axpy<T, false><<<G, kKLThreads, 0, st>>>(n1, a1.bP, in.kv1[l], part, G, ks, c->sc);
        }
        const T* b2 = band ? in.kb2[l] : a1.bP;
        down(l, kb);
        cycle(l + 1);
        up(l, band ? b2 : nullptr, take(l));
        k_kl_dots<T, 1><<<G, kKLThreads, 0, st>>>(v1.nx, v1.ny, v1.m, v1.We, v1.Wn, a1.xP, b2, in.kc1[l],
                                                  in.kv1[l], part, c->sc);
        if (parent_band) {
            if (!fold) k_kl_reduce<1><<<1, kRedThreads, 0, st>>>(part, G, ks, c->sc, single);
            BandKL<T> ke{};
            ke.v = in.kc1[l];
            ke.part = fold ? part : nullptr;
            ke.G = G;
            ke.ks = ks;
            ke.single = single;
            pend[l - 1] = ke;
        } else if (fold) {
            k_kl_combine<T, true><<<G, kKLThreads, 0, st>>>(n1, a1.xP, in.kc1[l], part, G, ks, c->sc, single);
        } else {
            k_kl_reduce<1><<<1, kRedThreads, 0, st>>>(part, G, ks, c->sc, single);
            k_kl_combine<T, false><<<G, kKLThreads, 0, st>>>(n1, a1.xP, in.kc1[l], part, G, ks, c->sc, single);
        }
    };
    cycle(0);
}

template <typename T>
void enqueue_vcycle_point(fld_ctx* c, Inner<T>& in, hipStream_t st) {
    const int L = (int)in.lv.size();
    const T omega = T(1);
    for (int l = 0; l < L - 1; ++l) {
        LevelT<T>& a = in.lv[l];
        LevelT<T>& b = in.lv[l + 1];
        k_pre_point<T><<<tile_grid(a.nx, a.ny), blk2d(), 0, st>>>(a.nx, a.ny, a.bP, a.m, a.We, a.Wn, a.xQ, b.bP, b.nx,
                                                                  b.ny, c->sc);
    }
    (void)join_setup(c, st);
    coarse_solve<T>(c, in, st);
    for (int l = L - 2; l >= 0; --l) {
        LevelT<T>& a = in.lv[l];
        LevelT<T>& b = in.lv[l + 1];
        if (l == 0) {
            const dim3 g = tile_grid(a.nx, a.ny);
            k_post_point<T, true><<<g, blk2d(), 0, st>>>(a.nx, a.ny, a.bP, a.m, a.We, a.Wn, a.xQ, b.xP, b.nx, omega,
                                                         a.xP, c->part_rz, c->sc);
            c->nrz = (int)(g.x * g.y);
        } else
            k_post_point<T, false><<<tile_grid(a.nx, a.ny), blk2d(), 0, st>>>(a.nx, a.ny, a.bP, a.m, a.We, a.Wn, a.xQ,
                                                                              b.xP, b.nx, omega, a.xP, c->part, c->sc);
    }
}

template <typename T>
void enqueue_vcycle(fld_ctx* c, Inner<T>& in, hipStream_t st) {
    if (in.lv.size() == 1) {
        if (c->sweeps_only) return;
        (void)join_setup(c, st);
        LevelT<T>& l0 = in.lv[0];
        if (in.dense) {
            const int n = l0.nx * l0.ny, G = (n + kDenseRows - 1) / kDenseRows;
            k_dense_solve<T, true><<<G, kDenseThreads, 0, st>>>(in.dg, in.Ainv, l0.bP, l0.xP, c->part_rz, c->sc);
            c->nrz = G;
        } else {
            k_coarse_solve<T, true><<<1, kCoarseSolveThreads, 0, st>>>(l0.nx * l0.ny, in.Ainv, l0.bP, l0.xP,
                                                                        c->part_rz, c->sc);
            c->nrz = 1;
        }
        return;
    }
    if (is_line(c->opt)) enqueue_vcycle_line<T>(c, in, st);
    else enqueue_vcycle_point<T>(c, in, st);
}

// Reliable update (only acts when the device flag `pending` is set, or when
// forced at the start of a solve): true FP64 residual of E + corr x, its norms
// and the convergence decision, then E += corr x and the re-scaled inner
// residual.
template <typename T>
void enqueue_check(fld_ctx* c, Inner<T>& in, double* E, int force, hipStream_t st) {
    const int nx = c->nx, ny = c->ny, n = nx * ny;
    const dim3 tg = tile_grid(nx, ny);
    k_resid64<T><<<tg, blk2d(), 0, st>>>(c->met, E, in.x, c->We, c->Wn, c->m, c->rhs, c->s, c->r64, c->part,
                                         c->part2, update_grid(n), c->sc, force);
    k_reduce_resid<<<1, kRedThreads, 0, st>>>(c->part, (int)(tg.x * tg.y), c->mu, c->sc, force);
    k_apply<T><<<grid1d(n), 256, 0, st>>>(n, E, c->r64, in.r, in.x, c->sc);
}

// One CG iteration ("slot"); `par` selects the p buffer pair (iterations
// alternate between the two).  E is the FP64 solution being refined.
template <typename T>
void enqueue_slot(fld_ctx* c, Inner<T>& in, int par, double* E, hipStream_t st) {
    const int nx = c->nx, ny = c->ny, n = nx * ny;
    LevelT<T>& l0 = in.lv[0];
    const dim3 tg = tile_grid(nx, ny);
    const int ntiles = (int)(tg.x * tg.y), nb1 = update_grid(n);
    // r.z: summed by every SpMV workgroup from the sweep's partials when they
    // are few, else once by one workgroup (c5's 4096-cell lines leave 2048,
    // whose re-summing cost the SpMV a third of its time)
    // (and, for the flexible beta, r_k+1 . z_k from k_update's partials)
    const bool flex = c->flex;
    const bool many_rz = c->nrz > 512 || flex;
    if (many_rz)
        k_reduce_rz<<<1, kRedThreads, 0, st>>>(c->part_rz, c->nrz, flex ? c->part_rzo : nullptr, nb1, c->rz_sum,
                                               c->sc);
    k_spmv<T><<<tg, blk2d(), 0, st>>>(nx, ny, l0.xP, in.p[par], in.p[par ^ 1], in.q, l0.m, l0.We, l0.Wn,
                                      many_rz ? c->rz_sum : c->part_rz, many_rz ? 1 : c->nrz,
                                      flex ? c->rz_sum + 1 : nullptr, c->part, c->sc);
    // alpha: summed inside k_update from the SpMV partials when they are few,
    // by one reduction workgroup otherwise
    const bool fold = ntiles <= 1024;
    if (!fold) k_reduce_pq<<<1, kRedThreads, 0, st>>>(c->part, ntiles, c->sc);
    // z_k (read by k_spmv above) stays in l0.xP until the next cycle
    k_update<T><<<nb1, 256, 0, st>>>(n, in.x, in.r, in.p[par ^ 1], in.q, c->part, fold ? ntiles : 0, c->part2,
                                     flex ? (const T*)l0.xP : nullptr, c->part_rzo, c->sc);
    enqueue_check<T>(c, in, E, 0, st);
    enqueue_vcycle<T>(c, in, st);
}

template <typename T>
fld_status build_hierarchy(fld_ctx* c, hipStream_t st) {
    Inner<T>& in = inner<T>(c);
    if (join_setup(c, st) != FLD_OK) return FLD_EHIP;
    const int L = (int)in.lv.size();
    const double omega = c->opt.mg_coarse_op == FLD_MG_HALVED ? 0.5 : 1.0;
    const bool line = is_line(c->opt);
    // the FP64 coarsening chain first: the coarsest level's inverse, built on
    // the side stream, then runs beside the inner-precision copies below
    // instead of after them (its ~50 us otherwise stalled the first V-cycle)
    for (int l = 1; l < L; ++l) {
        Level64& a = c->h64[l - 1];
        Level64& b = c->h64[l];
        k_coarsen<<<cell_grid(b.nx, b.ny), blk2d(), 0, st>>>(a.nx, a.ny, a.m, a.We, a.Wn, b.nx, b.ny, b.m, b.We, b.Wn,
                                                             omega);
    }
    Level64& cl = c->h64[L - 1];
    {
        // the coarsest inverse (one workgroup, ~40-240 us, up to kCoarseMax
        // cells; the block cyclic reduction, ~0.2-0.9 ms, above): it runs
        // beside the copies below, the prologue and the first down-leg of
        // the V-cycle, which do not need the inverse
        fld_ctx* ctx = c;
        HIPCHK(hipEventRecord(c->setup_fork, st));
        HIPCHK(hipStreamWaitEvent(c->setup_stream, c->setup_fork, 0));
        hipStream_t ss = c->setup_stream;
        const int w = std::min(cl.nx, cl.ny), tr = in.lv[L - 1].tr ? 1 : 0;
        if (in.dense) {
            // block cyclic reduction: staged coefficients, the level-0 line
            // blocks, the reduction up to one line, its inverse, the
            // back-substitution down to level 0 (the last level also writes
            // the inner-precision copy when that is a separate array)
            const DenseGeom& g = in.dg;
            const int n = g.w * g.nb, w = g.w, nn = g.w * g.w;
            k_dense_stage<<<(n + 255) / 256, 256, 0, ss>>>(g, in.dd, in.aa, in.cc);
            T* Gsep = std::is_same<T, double>::value ? nullptr : in.Ainv;
            auto run = [&](auto Wc) {
                constexpr int W = decltype(Wc)::value, TS = W / 16;
                constexpr size_t lds = dn_lds_bytes<W>();
                std::vector<int> Ns, offs;
                int N = g.nb, off = 0, l = 0;
                for (; N > 1; ++l) {
                    const int nx = (l + 1) & 1;
                    if (l == 0) {
                        // tridiagonal lines: Thomas solves and scalings, level 1
                        // straight from the staged coefficients (A^-1 of the odd
                        // lines in rAinv, transposed in rEt)
                        k_bcr_level0<W><<<N, 128, 0, ss>>>(
                            w, N, in.dd, in.aa, in.cc, in.rAinv, in.rEt, in.rA[nx], in.rC[nx], in.rCt[nx]);
                    } else {
                        const double *A = in.rA[l & 1], *C = in.rC[l & 1], *Ct = in.rCt[l & 1];
                        k_bcr_elim<W, TS><<<N / 2, 256, lds, ss>>>(w, N, A, C, Ct, in.rAinv + (size_t)off * nn,
                                                                   in.rE + (size_t)off * nn, in.rF + (size_t)off * nn,
                                                                   in.rEt + (size_t)off * nn,
                                                                   in.rFt + (size_t)off * nn);
                        k_bcr_reduce<W, TS><<<(N + 1) / 2, 256, lds, ss>>>(
                            w, N, A, C, Ct, in.rE + (size_t)off * nn, in.rF + (size_t)off * nn, in.rA[nx], in.rC[nx],
                            in.rCt[nx]);
                    }
                    Ns.push_back(N);
                    offs.push_back(off);
                    off += N / 2;
                    N = (N + 1) / 2;
                }
                k_bcr_top<W, TS><<<1, 256, 0, ss>>>(w, n, in.rA[l & 1], in.Gw);
                for (int lv = l - 1; lv >= 0; --lv) {
                    const int Nl = Ns[lv], o = offs[lv], sg = 1 << lv;
                    T* G = lv == 0 ? Gsep : nullptr;
                    const double *Ai = in.rAinv + (size_t)o * nn, *Et = in.rEt + (size_t)o * nn,
                                 *Ft = in.rFt + (size_t)o * nn;
                    const dim3 oe(Nl / 2, (Nl + 1) / 2), oo(Nl / 2, Nl / 2);
                    if (lv == 0) {
                        k_bcr_back<T, W, TS, true, true><<<oe, 256, lds, ss>>>(w, Nl, sg, n, Ai, Et, Ft, in.cc, in.Gw, G);
                        k_bcr_back<T, W, TS, false, true><<<oo, 256, lds, ss>>>(w, Nl, sg, n, Ai, Et, Ft, in.cc, in.Gw,
                                                                               G);
                    } else {
                        k_bcr_back<T, W, TS, true, false><<<oe, 256, lds, ss>>>(w, Nl, sg, n, Ai, Et, Ft, in.cc, in.Gw,
                                                                               G);
                        k_bcr_back<T, W, TS, false, false><<<oo, 256, lds, ss>>>(w, Nl, sg, n, Ai, Et, Ft, in.cc,
                                                                                in.Gw, G);
                    }
                }
            };
            if (w <= 32)
                run(std::integral_constant<int, 32>{});
            else
                run(std::integral_constant<int, 64>{});
        } else if (w <= 4)
            k_coarse_setup<T, 4><<<1, kCoarseMax, 0, ss>>>(cl.nx, cl.ny, tr, cl.m, cl.We, cl.Wn, c->mu, in.Ywork,
                                                           in.Ainv);
        else if (w <= 8)
            k_coarse_setup<T, 8><<<1, kCoarseMax, 0, ss>>>(cl.nx, cl.ny, tr, cl.m, cl.We, cl.Wn, c->mu, in.Ywork,
                                                           in.Ainv);
        else
            k_coarse_setup<T, kCoarseBand><<<1, kCoarseMax, 0, ss>>>(cl.nx, cl.ny, tr, cl.m, cl.We, cl.Wn, c->mu,
                                                                     in.Ywork, in.Ainv);
        HIPCHK(hipEventRecord(c->setup_join, ss));
        c->setup_pending = true;
    }
    for (int l = 0; l < L; ++l) {
        Level64& b = c->h64[l];
        LevelT<T>& lt = in.lv[l];
        const int n = b.nx * b.ny;
        k_demote_level<T><<<grid1d(n), 256, 0, st>>>(n, b.m, b.We, b.Wn, c->mu, lt.m, lt.We, lt.Wn);
        if (line && L > 1) {
            // transposed view: rows are the columns, east couplings are the north ones
            dim3 g((b.nx + kTT - 1) / kTT, (b.ny + kTT - 1) / kTT), blk(kTT, 8);
            k_transpose<T, 3><<<g, blk, 0, st>>>(b.nx, b.ny, lt.m, lt.Wn, lt.We, lt.mT, lt.WeT, lt.WnT, nullptr);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        c->err = std::string("hierarchy launch: ") + hipGetErrorString(e);
        return FLD_EHIP;
    }
    return FLD_OK;
}

template <typename T>
fld_status alloc_inner(fld_ctx* ctx) {
    Inner<T>& in = inner<T>(ctx);
    const size_t n = (size_t)ctx->nx * ctx->ny;
    const bool line = is_line(ctx->opt);
    in.lv.resize(ctx->h64.size());
    for (size_t l = 0; l < ctx->h64.size(); ++l) {
        LevelT<T>& lv = in.lv[l];
        lv.nx = ctx->h64[l].nx;
        lv.ny = ctx->h64[l].ny;
        lv.tr = line && (l & 1);
        const size_t m = (size_t)lv.nx * lv.ny;
        HIPCHK(ctx->alloc(&lv.m, m));
        HIPCHK(ctx->alloc(&lv.We, m));
        HIPCHK(ctx->alloc(&lv.Wn, m));
        if (line) {
            HIPCHK(ctx->alloc(&lv.mT, m));
            HIPCHK(ctx->alloc(&lv.WeT, m));
            HIPCHK(ctx->alloc(&lv.WnT, m));
            HIPCHK(ctx->alloc(&lv.bQ, m));
            HIPCHK(ctx->alloc(&lv.xQ2, m));
            HIPCHK(ctx->alloc(&lv.xPT, m));
        }
        if (l > 0) HIPCHK(ctx->alloc(&lv.bP, m));
        HIPCHK(ctx->alloc(&lv.xP, m));
        HIPCHK(ctx->alloc(&lv.xQ, m));
    }
    const LevelT<T>& cl = in.lv.back();
    const size_t ncl = (size_t)cl.nx * cl.ny;
    HIPCHK(ctx->alloc(&in.Ainv, ncl * ncl));
    in.dense = ncl > (size_t)kCoarseMax;
    if (in.dense) {
        DenseGeom& g = in.dg;
        const Level64& c64 = ctx->h64.back();
        g.nx = cl.nx;
        g.ny = cl.ny;
        g.cols = cl.ny < cl.nx ? 1 : 0;
        g.w = std::min(cl.nx, cl.ny);
        g.nb = std::max(cl.nx, cl.ny);  // > kCoarseMax / kDenseW: at least two lines, so level 0 reduces
        g.tr = cl.tr ? 1 : 0;
        g.m = c64.m;
        g.We = c64.We;
        g.Wn = c64.Wn;
        g.mu = ctx->mu;
        HIPCHK(ctx->alloc(&in.dd, ncl));
        HIPCHK(ctx->alloc(&in.aa, ncl));
        HIPCHK(ctx->alloc(&in.cc, ncl));
        // the reduction's line blocks (two levels) and, per eliminated line
        // (fewer than nb over all levels), A^-1, E, F, E^T, F^T
        const size_t blocks = (size_t)g.nb * g.w * g.w;
        for (int i = 0; i < 2; ++i) {
            HIPCHK(ctx->alloc(&in.rA[i], blocks));
            HIPCHK(ctx->alloc(&in.rC[i], blocks));
            HIPCHK(ctx->alloc(&in.rCt[i], blocks));
        }
        HIPCHK(ctx->alloc(&in.rAinv, blocks));
        HIPCHK(ctx->alloc(&in.rE, blocks));
        HIPCHK(ctx->alloc(&in.rF, blocks));
        HIPCHK(ctx->alloc(&in.rEt, blocks));
        HIPCHK(ctx->alloc(&in.rFt, blocks));
        if constexpr (std::is_same<T, double>::value)
            in.Gw = in.Ainv;
        else
            HIPCHK(ctx->alloc(&in.Gw, ncl * ncl));
        auto lds_attr = [&](auto Wc) -> hipError_t {
            constexpr int W = decltype(Wc)::value, TS = W / 16;
            const int b = (int)dn_lds_bytes<W>();
            const void* fs[] = {(const void*)k_bcr_elim<W, TS>,
                                (const void*)k_bcr_reduce<W, TS>,
                                (const void*)k_bcr_back<T, W, TS, true, true>,
                                (const void*)k_bcr_back<T, W, TS, false, true>,
                                (const void*)k_bcr_back<T, W, TS, true, false>,
                                (const void*)k_bcr_back<T, W, TS, false, false>};
            for (const void* f : fs) {
                const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        };
        HIPCHK(g.w <= 32 ? lds_attr(std::integral_constant<int, 32>{}) : lds_attr(std::integral_constant<int, 64>{}));
    } else {
        HIPCHK(ctx->alloc(&in.Ywork, ncl * ncl));
    }
    HIPCHK(ctx->alloc(&in.r, n));
    HIPCHK(ctx->alloc(&in.x, n));
    HIPCHK(ctx->alloc(&in.p[0], n));
    HIPCHK(ctx->alloc(&in.p[1], n));
    HIPCHK(ctx->alloc(&in.q, n));
    in.kl_mask = 0;
    in.kc1.assign(in.lv.size(), nullptr);
    in.kv1.assign(in.lv.size(), nullptr);
    in.kb2.assign(in.lv.size(), nullptr);
    if (line && (ctx->opt.mg_cycle == FLD_MG_CYCLE_KL_K || ctx->opt.mg_cycle == FLD_MG_CYCLE_KL_W2)) {
        // every second level from level 1 (levels 1, 3, 5, ...; a bit only
        // acts on a launched level, one above the LDS sub-cycle set below)
        for (size_t l = 1; l + 1 < in.lv.size() && l < 32; l += 2) {
            in.kl_mask |= 1u << l;
            const size_t n1 = (size_t)in.lv[l].nx * in.lv[l].ny;
            HIPCHK(ctx->alloc(&in.kc1[l], n1));
            HIPCHK(ctx->alloc(&in.kv1[l], n1));
            HIPCHK(ctx->alloc(&in.kb2[l], n1));
        }
    }
    in.lv[0].bP = in.r;  // the V-cycle's fine right-hand side is the CG residual
    // one-workgroup coarse sub-cycle: the finest level l >= 1 from which all
    // coarser levels fit in LDS (5 arrays each; the K-cycle adds two arrays of
    // level l and its partials) and whose lines fit one wavefront
    const int L = (int)in.lv.size();
    const bool kcyc = ctx->opt.mg_cycle != FLD_MG_CYCLE_V;
    constexpr int kRedSlots = 4 * (kSubThreads<T> / 64);
    in.sub_first = -1;
    int dev = 0, lds_max = 65536;
    HIPCHK(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        lds_max = 65536;
    if (line && L >= 3 && !in.dense) {
        for (int l = 1; l < L - 1 && in.sub_first < 0; ++l) {
            if (L - l > kSubMaxLevels) continue;
            if (std::max(in.lv[l].nx, in.lv[l].ny) > 64 * kLineMaxL) continue;
            size_t need = 0;
            for (int k = l; k < L; ++k) need += 5 * (size_t)(in.lv[k].nx + 1) * in.lv[k].ny;
            need += (size_t)in.lv[L - 1].nx * in.lv[L - 1].ny;  // coarsest right-hand side, gathered
            need += kSubThreads<T>;                              // coarsest solve's partial sums
            if (kcyc) need += 2 * (size_t)(in.lv[l].nx + 1) * in.lv[l].ny + kRedSlots;
            need *= sizeof(T);
            if (need <= (size_t)lds_max) {
                in.sub_first = l;
                in.sub_lds = need;
            }
        }
        if (in.sub_first > 0) {
            SubCycle<T>& S = in.sub;
            S.nlev = L - in.sub_first;
            int off = 0;
            for (int k = 0; k < S.nlev; ++k) {
                const LevelT<T>& lv = in.lv[in.sub_first + k];
                const int pitch = lv.nx + 1;
                S.lv[k] = SubLevel<T>{lv.nx, lv.ny, lv.m, lv.We, lv.Wn, off, lv.tr ? 1 : 0, pitch, pitch * lv.ny};
                off += 5 * pitch * lv.ny;
            }
            S.Ainv = in.Ainv;
            S.bc_off = off;
            S.part_off = off + in.lv[L - 1].nx * in.lv[L - 1].ny;
            const int mc = ctx->opt.mg_cycle;
            S.kcyc = (mc == FLD_MG_CYCLE_K || mc == FLD_MG_CYCLE_KL_K) ? 1
                     : (mc == FLD_MG_CYCLE_W2 || mc == FLD_MG_CYCLE_KL_W2) ? 2 : 0;
            S.k_off = S.part_off + kSubThreads<T>;
            if (in.sub_lds > 65536)
                HIPCHK(hipFuncSetAttribute((const void*)k_subcycle<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)in.sub_lds));
        }
    }
    // band-fused sweeps on the launched levels whose bands fit in LDS: band
    // height R (even, <= 8) as large as keeps >= 256 workgroups
    if (ctx->opt.smoother == FLD_SMOOTH_LINE) {
        const int Ld = in.sub_first > 0 ? in.sub_first : L - 1;
        size_t need_max = 0;
        auto pick = [&](int na, int rows, bool with_b) {
            for (int R = 8; R >= 2; R -= 2) {
                if (R > 2 && (rows + R - 1) / R < std::min(256, (rows + 1) / 2)) continue;
                const size_t need = band_lds_bytes<T>(na, R, with_b);
                if (need <= (size_t)lds_max) {
                    need_max = std::max(need_max, need);
                    return R;
                }
            }
            return 0;
        };
        for (int l = 0; l < Ld; ++l) {
            LevelT<T>& lv = in.lv[l];
            const int pnx = lv.tr ? lv.ny : lv.nx, pny = lv.tr ? lv.nx : lv.ny;
            // rows so long that even 4-row bands overflow LDS leave one
            // workgroup per CU: such levels are bandwidth-bound and run faster
            // with the one-launch-per-half-sweep kernels (measured on 4096-cell
            // rows: 462 us against 260 us per level visit)
            const bool roomy = band_lds_bytes<T>(pnx, 4, true) <= (size_t)lds_max &&
                               band_lds_bytes<T>(pny, 4, false) <= (size_t)lds_max;
            const int Rp = roomy ? pick(pnx, pny, true) : 0, Rq = roomy ? pick(pny, pnx, false) : 0;
            lv.band = Rp > 0 && Rq > 0;
            lv.Rp = Rp;
            lv.Rq = Rq;
        }
        if (need_max > 65536) {
            const int sz = (int)need_max;
            const void* fns[] = {
                (const void*)k_band<T, kLineMaxL, LINE_ZERO, 0, true, true, false>,
                (const void*)k_band<T, kLineMaxL, LINE_NORMAL, 0, false, false, false>,
                (const void*)k_band<T, kLineMaxL, LINE_PROLONG, 1, true, false, false>,
                (const void*)k_band<T, kLineMaxL, LINE_NORMAL, 1, false, false, true>,
                (const void*)k_band<T, kLineMaxL, LINE_NORMAL, 1, false, false, false>};
            for (const void* f : fns) HIPCHK(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, sz));
        }
    }
    HIPCHK(hipMemset(in.r, 0, sizeof(T) * n));
    HIPCHK(hipMemset(in.x, 0, sizeof(T) * n));
    HIPCHK(hipMemset(in.p[0], 0, sizeof(T) * n));
    HIPCHK(hipMemset(in.p[1], 0, sizeof(T) * n));
    return FLD_OK;
}

void fill_info(fld_ctx* c, fld_solve_info* info, int status, float ms) {
    if (!info) return;
    const Scalars& s = *c->hsc;
    info->status = status;
    info->outer_iters = s.nchecks;
    info->inner_iters = s.iter;
    info->mg_levels = (int)c->h64.size();
    info->rel_resid = s.rel_sel;
    info->rel_resid_row = s.rel_row;
    info->rel_resid_scaled = s.rel_scaled;
    info->ms = ms;
}

// Captures `chunk` CG iterations (an even number, so the p buffers line up)
// into a hipGraph on a private stream; re-captured only when the solution
// pointer changes.  The graph holds kernel nodes only.
template <typename T>
fld_status capture_chunk(fld_ctx* ctx, Inner<T>& in, double* E, int chunk) {
    if (in.chunk_exec && in.chunk_E == E && in.chunk_len == chunk) return FLD_OK;
    if (in.chunk_exec) {
        HIPCHK(hipGraphExecDestroy(in.chunk_exec));
        in.chunk_exec = nullptr;
    }
    if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < chunk; ++k) enqueue_slot<T>(ctx, in, k & 1, E, ctx->cap_stream);
    hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (e != hipSuccess) {
        ctx->err = std::string("graph capture: ") + hipGetErrorString(e);
        return FLD_EHIP;
    }
    e = hipGraphInstantiate(&in.chunk_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        in.chunk_exec = nullptr;
        ctx->err = std::string("graph instantiate: ") + hipGetErrorString(e);
        return FLD_EHIP;
    }
    in.chunk_E = E;
    in.chunk_len = chunk;
    return FLD_OK;
}

// CG iterations as launches of the captured chunk graph (chunk slots each),
// the solver state copied after every launch to one of two pinned mirrors.
// While the predicted iteration count (the last solve's, 0 if unknown) lies
// beyond the chunk being waited for, the next chunk is queued before the host
// reads that chunk's flags, so the GPU does not idle on the host; near the
// predicted end the host reads first and queues only what is still needed,
// so no chunk of early-exit slots is left to run.  Returns false on a HIP
// error.
template <typename T>
bool run_chunks(fld_ctx* ctx, Inner<T>& in, int chunk, int max_iter, int predict, hipStream_t st) {
    Scalars* mirror[2] = {ctx->hsc, ctx->hsc2};
    const int max_chunks = (max_iter + chunk - 1) / chunk + 1;
    auto launch = [&](int c) -> bool {
        return hipGraphLaunch(in.chunk_exec, st) == hipSuccess &&
               hipMemcpyAsync(mirror[c & 1], ctx->sc, sizeof(Scalars), hipMemcpyDeviceToHost, st) == hipSuccess &&
               hipEventRecord(ctx->pev[c & 1], st) == hipSuccess;
    };
    if (!launch(0)) return false;
    int queued = 1;
    for (int c = 0;; ++c) {
        if (queued == c + 1 && c + 1 < max_chunks && predict > (c + 1) * chunk) {
            if (!launch(c + 1)) return false;
            ++queued;
        }
        if (hipEventSynchronize(ctx->pev[c & 1]) != hipSuccess) return false;
        if (mirror[c & 1]->done || c + 1 >= max_chunks) {
            ctx->last_iters = mirror[c & 1]->iter;
            return true;
        }
        if (queued == c + 1) {
            if (!launch(c + 1)) return false;
            ++queued;
        }
    }
}

template <typename T>
fld_status solve_impl(fld_ctx* ctx, double* E, fld_solve_info* info) {
    auto t0 = std::chrono::steady_clock::now();
    Inner<T>& in = inner<T>(ctx);
    hipStream_t st = ctx->stream;
    const int nx = ctx->nx, ny = ctx->ny, n = nx * ny;
    const fld_options& o = ctx->opt;
    const bool fp32only = o.precision == FLD_FP32;
    const bool mixed = o.precision == FLD_MIXED;
    // true-residual check once the binary32 recurrence residual has fallen 100x
    // (10x checked twice as often for the same iteration count: c2 -2 %)
    const double delta = mixed ? 0.01 : 1e-3;
    const int max_iter = o.max_inner;
    k_init_scalars<<<1, 1, 0, st>>>(ctx->sc, o.rel_tol, delta * delta, o.inner_rtol * o.inner_rtol, max_iter, o.norm,
                                    fp32only ? 0 : 1);
    // prologue: true residual of the initial guess, inner residual, first V-cycle
    enqueue_check<T>(ctx, in, E, 1, st);
    enqueue_vcycle<T>(ctx, in, st);
    HIPCHK(hipGetLastError());
    const int chunk = o.chunk;
    // events recorded inside a captured graph cannot be timed on this runtime,
    // so measured solves queue plain launches
    const bool graph = o.use_graph != 0 && !ctx->prof.on;
    if (graph) {
        // captured chunks, read ahead while the last solve's iteration count
        // says more are needed (run_chunks); a non-finite input is reported
        // after the solve
        fld_status gs = capture_chunk<T>(ctx, in, E, chunk);
        if (gs != FLD_OK) return gs;
        if (!run_chunks<T>(ctx, in, chunk, max_iter, ctx->last_iters, st)) {
            ctx->err = "solve: chunk launch or flag read failed";
            return FLD_EHIP;
        }
    } else {
        HIPCHK(hipMemcpyAsync(ctx->hsc, ctx->sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(ctx->herr, ctx->err_flag, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (*ctx->herr) {
            ctx->err = "non-finite or out-of-domain input field";
            fill_info(ctx, info, FLD_ENONFINITE, 0.f);
            return FLD_ENONFINITE;
        }
        if (prof_harvest(ctx) != FLD_OK) return FLD_EHIP;
        int launched = 0;
        while (!ctx->hsc->done && launched < max_iter + chunk) {
            for (int k = 0; k < chunk; ++k) enqueue_slot<T>(ctx, in, (launched + k) & 1, E, st);
            launched += chunk;
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(ctx->hsc, ctx->sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            if (prof_harvest(ctx) != FLD_OK) return FLD_EHIP;
        }
    }
    k_correct<T><<<grid1d(n), 256, 0, st>>>(n, E, in.x, ctx->sc, 1, ctx->err_flag);
    HIPCHK(hipMemcpyAsync(ctx->hsc, ctx->sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ctx->herr, ctx->err_flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (*ctx->herr) {
        ctx->err = "non-finite or out-of-domain input field";
        fill_info(ctx, info, FLD_ENONFINITE, 0.f);
        return FLD_ENONFINITE;
    }
    int status = ctx->hsc->status;
    if (status == ST_OK && !ctx->hsc->done) status = FLD_ENOCONV;
    const float ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    fill_info(ctx, info, status, ms);
    if (status != FLD_OK) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "solve status %d after %d iterations, rel. residual %.3e", status,
                      ctx->hsc->iter, ctx->hsc->rel_sel);
        ctx->err = buf;
    }
    return (fld_status)status;
}

}  // namespace

namespace {

fld_status check_fields(fld_ctx* ctx, const double* E, const double* T, const double* rho, const double* kR,
                        const double* kP, const double* cv, const double* ghost, double dt) {
    if (!E || !T || !rho || !kR || !kP || !cv) { ctx->err = "null field pointer"; return FLD_EINVAL; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { ctx->err = "dt must be > 0"; return FLD_EINVAL; }
    for (int sd = 0; sd < 4; ++sd)
        if (ctx->bc.kind[sd] == BC_DIRICHLET_GHOST && !ghost) { ctx->err = "ghost_E required"; return FLD_EINVAL; }
    return FLD_OK;
}

// Assembly and multigrid hierarchy, kernels only (capturable).
// Eop: the E the face coefficients and the advection term are taken from
// (null: E; a sub-cycled step passes its saved E^n).
fld_status enqueue_assemble(fld_ctx* ctx, const double* E, const double* T, const double* rho, const double* kR,
                            const double* kP, const double* cv, const double* ghost, double dt, hipStream_t st,
                            const double* Eop = nullptr) {
    k_zero_int<<<1, 1, 0, st>>>(ctx->err_flag);
    if (ctx->cv_p != 0.0) {
        // c_v(T^n) of the power law; the gas update reads the same values
        const int n = ctx->nx * ctx->ny;
        k_cv_law<<<grid1d(n), 256, 0, st>>>(n, cv, T, 1.0 / ctx->cv_Tref, ctx->cv_p, ctx->cvl);
        cv = ctx->cvl;
    }
    AsmIn in{E, T, rho, kR, kP, cv, ghost, dt, ctx->opt.limiter, ctx->bc, ctx->fx, ctx->fy, Eop};
    AsmOut out{ctx->We, ctx->Wn, ctx->m, ctx->rhs, ctx->s, ctx->err_flag, ctx->part, ctx->bside, ctx->rside};
    const dim3 ag = cell_grid(ctx->nx, ctx->ny);
    k_assemble<<<ag, blk2d(), 0, st>>>(ctx->met, in, out);
    k_reduce_max<<<1, kRedThreads, 0, st>>>(ctx->part, (int)(ag.x * ag.y), ctx->mu);
    HIPCHK(hipGetLastError());
    fld_status s = inner_is_float(ctx) ? build_hierarchy<float>(ctx, st) : build_hierarchy<double>(ctx, st);
    if (s != FLD_OK) return s;
    ctx->T = T;
    ctx->rho = rho;
    ctx->kP = kP;
    ctx->cv = cv;
    ctx->dt = dt;
    return FLD_OK;
}

// A solve with a fixed budget of `slots` CG iterations and device-side early
// exit, then the final correction (capturable: no host synchronisation).
template <typename T>
void enqueue_solve_fixed(fld_ctx* ctx, double* E, int slots, hipStream_t st) {
    Inner<T>& in = inner<T>(ctx);
    const fld_options& o = ctx->opt;
    const int n = ctx->nx * ctx->ny;
    const double delta = o.precision == FLD_MIXED ? 0.01 : 1e-3;
    k_init_scalars<<<1, 1, 0, st>>>(ctx->sc, o.rel_tol, delta * delta, o.inner_rtol * o.inner_rtol, slots, o.norm,
                                    o.precision == FLD_FP32 ? 0 : 1);
    enqueue_check<T>(ctx, in, E, 1, st);
    enqueue_vcycle<T>(ctx, in, st);
    for (int k = 0; k < slots; ++k) enqueue_slot<T>(ctx, in, k & 1, E, st);
    k_correct<T><<<grid1d(n), 256, 0, st>>>(n, E, in.x, ctx->sc, 1, ctx->err_flag);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

void fld_default_options(fld_options* o) {
    if (!o) return;
    o->precision = FLD_MIXED;
    o->limiter = FLD_LIMITER_LP;
    o->norm = FLD_NORM_ROW;
    o->rel_tol = 1e-10;
    o->max_outer = 8;
    o->max_inner = 2000;
    o->inner_rtol = 1e-5;
    o->mg_coarse_max = 64;
    o->mg_coarse_op = FLD_MG_HALVED;
    o->smoother = FLD_SMOOTH_LINE;
    o->chunk = 8;
    o->use_graph = 1;
    o->mg_cycle = FLD_MG_CYCLE_K;
}

const char* fld_version(void) { return kVersion; }

const char* fld_status_string(fld_status s) {
    switch (s) {
        case FLD_OK: return "ok";
        case FLD_EINVAL: return "invalid argument";
        case FLD_ENOMEM: return "out of device memory";
        case FLD_EHIP: return "HIP runtime error";
        case FLD_ENOCONV: return "tolerance not reached";
        case FLD_EBREAKDOWN: return "CG breakdown";
        case FLD_ENONFINITE: return "non-finite or out-of-domain input";
        case FLD_ENOTREADY: return "not assembled";
    }
    return "unknown status";
}

const char* fld_last_error(const fld_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t fld_mg_levels(const fld_ctx* ctx) { return ctx ? (int32_t)ctx->h64.size() : 0; }

fld_status fld_profile(fld_ctx* ctx, int32_t enable) {
    if (!ctx) return FLD_EINVAL;
    auto& P = ctx->prof;
    if (enable && P.slots == 0) {
        // one chunk of iterations plus the first V-cycle of a solve
        const int per_vcycle = 8 * (int)ctx->h64.size() + 8;
        P.slots = per_vcycle * (ctx->opt.chunk + 1);
        P.ev.resize(2 * P.slots);
        for (auto& e : P.ev) HIPCHK(hipEventCreate(&e));
        P.bytes.assign(P.slots, 0.0);
        HIPCHK(ctx->alloc(&P.ran, (size_t)P.slots));
        HIPCHK(hipMemset(P.ran, 0, sizeof(int) * P.slots));
        HIPCHK(hipHostMalloc((void**)&P.hran, sizeof(int) * P.slots, hipHostMallocDefault));
    }
    P.on = enable != 0;
    P.used = 0;
    P.launches = 0;
    P.ms = 0.0;
    P.total_bytes = 0.0;
    return FLD_OK;
}

fld_status fld_profile_overhead(fld_ctx* ctx, int32_t reps, double* us_per_launch) {
    if (!ctx || reps < 1 || !us_per_launch) return FLD_EINVAL;
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    double tot = 0.0;
    for (int k = 0; k < reps; ++k) {
        HIPCHK(hipEventRecord(a, ctx->stream));
        k_noop<<<1, 64, 0, ctx->stream>>>(nullptr);
        HIPCHK(hipEventRecord(b, ctx->stream));
        HIPCHK(hipEventSynchronize(b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, a, b));
        tot += ms;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *us_per_launch = 1e3 * tot / reps;
    return FLD_OK;
}

fld_status fld_profile_sweeps(fld_ctx* ctx, int32_t reps, double* us_per_launch, double* floor_us,
                              double* bytes_per_launch, int32_t* launches) {
    return fld_profile_sweeps_range(ctx, 0, 0, reps, us_per_launch, floor_us, bytes_per_launch, launches);
}

fld_status fld_profile_sweeps_levels(fld_ctx* ctx, int32_t levels, int32_t reps, double* us_per_launch,
                                     double* floor_us, double* bytes_per_launch, int32_t* launches) {
    return fld_profile_sweeps_range(ctx, 0, levels, reps, us_per_launch, floor_us, bytes_per_launch, launches);
}

fld_status fld_profile_sweeps_range(fld_ctx* ctx, int32_t first, int32_t levels, int32_t reps,
                                    double* us_per_launch, double* floor_us, double* bytes_per_launch,
                                    int32_t* launches) {
    if (!ctx || reps < 1 || first < 0 || levels < 0 || !us_per_launch || !floor_us || !bytes_per_launch ||
        !launches)
        return FLD_EINVAL;
    if (!ctx->assembled) {
        ctx->err = "fld_profile_sweeps before fld_assemble";
        return FLD_ENOTREADY;
    }
    if (!is_line(ctx->opt)) {
        ctx->err = "fld_profile_sweeps needs a line smoother";
        return FLD_EINVAL;
    }
    // a context without graphs (use_graph = 0) replays the sweeps as plain
    // launches, so that counter tools that do not follow graphs see them
    const bool graph = ctx->opt.use_graph != 0;
    if (graph && !ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    struct Events {
        hipEvent_t a = nullptr, b = nullptr;
        ~Events() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    HIPCHK(hipEventCreate(&ev.a));
    HIPCHK(hipEventCreate(&ev.b));
    hipEvent_t a = ev.a, b = ev.b;
    // a solver state that is never done, so every sweep works
    k_init_scalars<<<1, 1, 0, ctx->stream>>>(ctx->sc_sweep, 1e-300, 0.0, 0.0, 1, 0, 1);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    Scalars* keep = ctx->sc;
    const bool prof_on = ctx->prof.on;
    const int nrz_keep = ctx->nrz;
    auto enter = [&]() {
        ctx->sc = ctx->sc_sweep;
        ctx->prof.on = false;
        ctx->sweeps_only = true;
        ctx->sweep_first = first;
        ctx->sweep_levels = levels;
    };
    auto leave = [&]() {
        ctx->sc = keep;
        ctx->prof.on = prof_on;
        ctx->sweeps_only = false;
        ctx->sweep_first = 0;
        ctx->sweep_levels = 0;
        ctx->nrz = nrz_keep;
    };
    auto sweeps = [&](hipStream_t st) {
        if (inner_is_float(ctx)) enqueue_vcycle<float>(ctx, ctx->i32, st);
        else enqueue_vcycle<double>(ctx, ctx->i64, st);
    };
    enter();
    ctx->sweep_launches = 0;
    ctx->sweep_bytes = 0.0;
    hipGraph_t g = nullptr;
    hipError_t e = hipSuccess;
    if (graph) {
        e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            sweeps(ctx->cap_stream);
            e = hipStreamEndCapture(ctx->cap_stream, &g);
        }
    } else {
        sweeps(ctx->stream);  // warm-up, and the launch count
        e = hipGetLastError();
    }
    const int nl = ctx->sweep_launches;
    const double nbytes = ctx->sweep_bytes;
    if (graph) leave();
    if (e != hipSuccess) {
        if (!graph) leave();
        ctx->err = std::string("sweep capture: ") + hipGetErrorString(e);
        return FLD_EHIP;
    }
    if (nl == 0) {
        if (graph) (void)hipGraphDestroy(g);
        else leave();
        ctx->err = "no line-sweep launch in the level range";
        return FLD_EINVAL;
    }
    hipGraphExec_t ge = nullptr, ge0 = nullptr;
    if (graph) {
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            ctx->err = std::string("sweep graph: ") + hipGetErrorString(e);
            return FLD_EHIP;
        }
        // the same number of empty launches, captured and replayed alike:
        // the graph's cost per dependent launch
        e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            for (int k = 0; k < nl; ++k) k_noop<<<1, 64, 0, ctx->cap_stream>>>(nullptr);
            e = hipStreamEndCapture(ctx->cap_stream, &g);
        }
        if (e == hipSuccess) {
            e = hipGraphInstantiate(&ge0, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
        }
        if (e != hipSuccess) {
            (void)hipGraphExecDestroy(ge);
            ctx->err = std::string("empty-launch graph: ") + hipGetErrorString(e);
            return FLD_EHIP;
        }
    }
    // one pass of the work (graph or plain launches), a warm-up pass first
    auto replay = [&](bool empty, float* ms) -> hipError_t {
        auto pass = [&]() -> hipError_t {
            if (graph) return hipGraphLaunch(empty ? ge0 : ge, ctx->stream);
            if (empty)
                for (int k = 0; k < nl; ++k) k_noop<<<1, 64, 0, ctx->stream>>>(nullptr);
            else
                sweeps(ctx->stream);
            return hipGetLastError();
        };
        hipError_t r = pass();
        if (r == hipSuccess) r = hipEventRecord(a, ctx->stream);
        for (int k = 0; k < reps && r == hipSuccess; ++k) r = pass();
        if (r == hipSuccess) r = hipEventRecord(b, ctx->stream);
        if (r == hipSuccess) r = hipEventSynchronize(b);
        if (r == hipSuccess) r = hipEventElapsedTime(ms, a, b);
        return r;
    };
    float ms = 0.f, ms0 = 0.f;
    e = replay(false, &ms);
    if (e == hipSuccess) e = replay(true, &ms0);
    if (!graph) leave();
    if (graph) {
        (void)hipGraphExecDestroy(ge);
        (void)hipGraphExecDestroy(ge0);
    }
    if (e != hipSuccess) {
        ctx->err = std::string("sweep replay: ") + hipGetErrorString(e);
        return FLD_EHIP;
    }
    *launches = nl;
    *us_per_launch = 1e3 * ms / ((double)reps * nl);
    *floor_us = 1e3 * ms0 / ((double)reps * nl);
    *bytes_per_launch = nbytes / nl;
    return FLD_OK;
}

fld_status fld_profile_read(fld_ctx* ctx, int64_t* launches, double* total_ms, double* bytes) {
    if (!ctx) return FLD_EINVAL;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (prof_harvest(ctx) != FLD_OK) return FLD_EHIP;
    if (launches) *launches = ctx->prof.launches;
    if (total_ms) *total_ms = ctx->prof.ms;
    if (bytes) *bytes = ctx->prof.total_bytes;
    return FLD_OK;
}

void fld_destroy(fld_ctx* ctx) {
    if (!ctx) return;
    // errors are ignored here: the context is being torn down either way
    if (ctx->i32.chunk_exec) (void)hipGraphExecDestroy(ctx->i32.chunk_exec);
    if (ctx->i64.chunk_exec) (void)hipGraphExecDestroy(ctx->i64.chunk_exec);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->setup_stream) (void)hipStreamSynchronize(ctx->setup_stream);
    for (void* p : ctx->allocs) (void)hipFree(p);
    if (ctx->hsc) (void)hipHostFree(ctx->hsc);
    if (ctx->herr) (void)hipHostFree(ctx->herr);
    if (ctx->hsc2) (void)hipHostFree(ctx->hsc2);
    for (hipEvent_t e : ctx->pev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->setup_stream) (void)hipStreamDestroy(ctx->setup_stream);
    if (ctx->setup_fork) (void)hipEventDestroy(ctx->setup_fork);
    if (ctx->setup_join) (void)hipEventDestroy(ctx->setup_join);
    if (ctx->cap_fork) (void)hipEventDestroy(ctx->cap_fork);
    if (ctx->cap_join) (void)hipEventDestroy(ctx->cap_join);
    for (auto& e : ctx->prof.ev) (void)hipEventDestroy(e);
    if (ctx->prof.hran) (void)hipHostFree(ctx->prof.hran);
    delete ctx;
}

fld_status fld_create(fld_ctx** out, const fld_grid* grid, const fld_options* opt, void* stream) {
    if (!out || !grid) return FLD_EINVAL;
    *out = nullptr;
    fld_ctx* ctx = new fld_ctx();
    auto fail = [&](fld_status s, const std::string& msg) {
        ctx->err = msg;
        *out = ctx;  // keep the context so fld_last_error works; caller destroys it
        return s;
    };
    if (opt) ctx->opt = *opt;
    else fld_default_options(&ctx->opt);
    std::string why;
    if (validate_options(&ctx->opt, why) != FLD_OK) return fail(FLD_EINVAL, "bad option: " + why);
    ctx->flex = is_line(ctx->opt) && ctx->opt.mg_cycle != FLD_MG_CYCLE_V;
    const int nx = grid->nx, ny = grid->ny;
    if (nx < 1 || ny < 1 || (int64_t)nx * ny > (int64_t(1) << 28)) return fail(FLD_EINVAL, "grid size");
    if (grid->geom != FLD_CARTESIAN && grid->geom != FLD_SPHERICAL_POLAR) return fail(FLD_EINVAL, "geometry");
    if (!grid->x_faces || !grid->y_faces) return fail(FLD_EINVAL, "face arrays");
    for (int i = 0; i < nx; ++i)
        if (!(grid->x_faces[i + 1] > grid->x_faces[i]) || !std::isfinite(grid->x_faces[i + 1]))
            return fail(FLD_EINVAL, "x faces must increase");
    for (int j = 0; j < ny; ++j)
        if (!(grid->y_faces[j + 1] > grid->y_faces[j]) || !std::isfinite(grid->y_faces[j + 1]))
            return fail(FLD_EINVAL, "y faces must increase");
    if (grid->geom == FLD_SPHERICAL_POLAR) {
        if (!(grid->x_faces[0] > 0.0)) return fail(FLD_EINVAL, "spherical radii must be > 0");
        if (grid->y_faces[0] < 0.0 || grid->y_faces[ny] > 3.14159265358979323846 + 1e-12)
            return fail(FLD_EINVAL, "theta faces must lie in [0, pi]");
    }
    for (int sd = 0; sd < 4; ++sd) {
        const int k = grid->bc[sd].kind;
        if (k < 0 || k > FLD_BC_MILNE) return fail(FLD_EINVAL, "boundary kind");
        if (k == FLD_BC_AXIS && (grid->geom != FLD_SPHERICAL_POLAR || sd < 2))
            return fail(FLD_EINVAL, "axis boundary needs a spherical theta side");
        if (k == FLD_BC_DIRICHLET_FACE && !(grid->bc[sd].value > 0.0)) return fail(FLD_EINVAL, "Dirichlet temperature");
        if (k == FLD_BC_FLUX_IN && !std::isfinite(grid->bc[sd].value)) return fail(FLD_EINVAL, "flux value");
        ctx->bc.kind[sd] = k;
        ctx->bc.value[sd] = grid->bc[sd].value;
    }
    ctx->nx = nx;
    ctx->ny = ny;
    ctx->geom = grid->geom;
    ctx->stream = static_cast<hipStream_t>(stream);
    const size_t n = (size_t)nx * ny;
    // device memory
#define ALLOC(p, cnt) \
    if (ctx->alloc(&(p), (cnt)) != hipSuccess) return fail(FLD_ENOMEM, "hipMalloc " #p)
    double *vx, *vy, *sx, *sy, *ax, *hxL, *hxR, *hyL, *hyR, *arc;
    ALLOC(ctx->xf, nx + 1);
    ALLOC(ctx->yf, ny + 1);
    ALLOC(vx, nx); ALLOC(ax, nx); ALLOC(arc, nx); ALLOC(sx, nx + 1); ALLOC(hxL, nx + 1); ALLOC(hxR, nx + 1);
    ALLOC(vy, ny); ALLOC(sy, ny + 1); ALLOC(hyL, ny + 1); ALLOC(hyR, ny + 1);
    ALLOC(ctx->We, n); ALLOC(ctx->Wn, n); ALLOC(ctx->m, n); ALLOC(ctx->rhs, n); ALLOC(ctx->s, n); ALLOC(ctx->r64, n);
    ctx->met = Metrics{nx, ny, vx, vy, sx, sy, ax, hxL, hxR, hyL, hyR, arc};
    // multigrid levels: 2x2 aggregation until at most mg_coarse_max cells; the
    // fine level is the assembled operator itself
    {
        int lx = nx, ly = ny;
        while (true) {
            Level64 L;
            L.nx = lx;
            L.ny = ly;
            if (ctx->h64.empty()) {
                L.m = ctx->m;
                L.We = ctx->We;
                L.Wn = ctx->Wn;
            } else {
                ALLOC(L.m, (size_t)lx * ly);
                ALLOC(L.We, (size_t)lx * ly);
                ALLOC(L.Wn, (size_t)lx * ly);
            }
            ctx->h64.push_back(L);
            if ((int64_t)lx * ly <= ctx->opt.mg_coarse_max) break;
            lx = (lx + 1) / 2;
            ly = (ly + 1) / 2;
        }
    }
    if (is_line(ctx->opt) && (nx > kLineWG * kLineMaxL || ny > kLineWG * kLineMaxL))
        return fail(FLD_EINVAL, "line smoother supports nx, ny <= 4096; use the point smoother");
    const size_t tiles = (size_t)tile_grid(nx, ny).x * tile_grid(nx, ny).y;
    ctx->npart = std::max<size_t>(tiles * 5, (size_t)k1DBlocksMax);
    ALLOC(ctx->part, ctx->npart);
    ALLOC(ctx->part2, (size_t)k1DBlocksMax);
    ALLOC(ctx->part_rz, ctx->npart);
    ALLOC(ctx->rz_sum, 2);
    ALLOC(ctx->part_rzo, (size_t)k1DBlocksMax);
    ALLOC(ctx->kpart, 3 * (size_t)kKLMaxWG * 32);
    ALLOC(ctx->kscal, 32);
    ALLOC(ctx->sc, 1);
    ALLOC(ctx->sc_sweep, 1);
    ALLOC(ctx->err_flag, 1);
    ALLOC(ctx->mu, 1);
    ALLOC(ctx->dt_lim, 1);
    ALLOC(ctx->bside, 2 * (size_t)(nx + ny));
    ALLOC(ctx->rside, 2 * (size_t)(nx + ny));
    ALLOC(ctx->Esave, n);
    ALLOC(ctx->Tsave, n);
    ALLOC(ctx->seg_info, kStepSeg);
    ALLOC(ctx->seg_count, 1);
#undef ALLOC
    if (hipHostMalloc((void**)&ctx->hsc, sizeof(Scalars), hipHostMallocDefault) != hipSuccess)
        return fail(FLD_ENOMEM, "pinned scalars");
    if (hipHostMalloc((void**)&ctx->herr, sizeof(int), hipHostMallocDefault) != hipSuccess)
        return fail(FLD_ENOMEM, "pinned flag");
    if (hipHostMalloc((void**)&ctx->hsc2, sizeof(Scalars), hipHostMallocDefault) != hipSuccess)
        return fail(FLD_ENOMEM, "pinned scalars");
    std::memset(ctx->hsc, 0, sizeof(Scalars));
    std::memset(ctx->hsc2, 0, sizeof(Scalars));
    if (hipEventCreateWithFlags(&ctx->pev[0], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->pev[1], hipEventDisableTiming) != hipSuccess)
        return fail(FLD_EHIP, "events");
    *ctx->herr = 0;
    if (hipStreamCreateWithFlags(&ctx->setup_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->setup_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->setup_join, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->cap_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ctx->cap_join, hipEventDisableTiming) != hipSuccess)
        return fail(FLD_EHIP, "set-up stream");
    fld_status s;
    if (inner_is_float(ctx)) s = alloc_inner<float>(ctx);
    else s = alloc_inner<double>(ctx);
    if (s != FLD_OK) return fail(s, ctx->err);
    if (hipMemset(ctx->sc, 0, sizeof(Scalars)) != hipSuccess) return fail(FLD_EHIP, "memset scalars");
    if (hipMemset(ctx->err_flag, 0, sizeof(int)) != hipSuccess) return fail(FLD_EHIP, "memset flag");
    if (hipMemcpy(ctx->xf, grid->x_faces, sizeof(double) * (nx + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(ctx->yf, grid->y_faces, sizeof(double) * (ny + 1), hipMemcpyHostToDevice) != hipSuccess)
        return fail(FLD_EHIP, "copy faces");
    const int mt = std::max(nx, ny) + 1;
    k_metrics<<<(mt + 255) / 256, 256, 0, ctx->stream>>>(ctx->geom, nx, ny, ctx->xf, ctx->yf, vx, vy, sx, sy, ax, hxL,
                                                         hxR, hyL, hyR, arc);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(ctx->stream) != hipSuccess)
        return fail(FLD_EHIP, "metrics kernel");
    *out = ctx;
    return FLD_OK;
}

fld_status fld_assemble(fld_ctx* ctx, const double* E, const double* T, const double* rho, const double* kR,
                        const double* kP, const double* cv, const double* ghost, double dt) {
    if (!ctx) return FLD_EINVAL;
    fld_status s = check_fields(ctx, E, T, rho, kR, kP, cv, ghost, dt);
    if (s != FLD_OK) return s;
    s = enqueue_assemble(ctx, E, T, rho, kR, kP, cv, ghost, dt, ctx->stream);
    if (s != FLD_OK) return s;
    ctx->assembled = true;
    return FLD_OK;
}

namespace {

fld_status solve_checked(fld_ctx* ctx, double* E, fld_solve_info* info) {
    if (!E) { ctx->err = "null E"; return FLD_EINVAL; }
    if (!ctx->assembled) { ctx->err = "fld_assemble first"; return FLD_ENOTREADY; }
    return inner_is_float(ctx) ? solve_impl<float>(ctx, E, info) : solve_impl<double>(ctx, E, info);
}

// Host-driven solves after a replayed multi-step graph are refused: on the
// 4096 x 2048 grid and on the 1024 x 1024 grid, runs of single steps on a
// context that had replayed fld_steps_graph's captured step ended with a host
// heap-corruption abort whose cause is not established.
fld_status refuse_after_replay(fld_ctx* ctx) {
    if (!ctx->replayed) return FLD_OK;
    ctx->err = "this context has replayed a captured multi-step graph (fld_steps_graph); it serves further "
               "fld_steps_graph calls only: use another context for single steps";
    return FLD_EINVAL;
}

}  // namespace

fld_status fld_solve(fld_ctx* ctx, double* E, fld_solve_info* info) {
    if (!ctx) return FLD_EINVAL;
    fld_status g = refuse_after_replay(ctx);
    if (g != FLD_OK) return g;
    return solve_checked(ctx, E, info);
}

fld_status fld_gas_update(fld_ctx* ctx, const double* E, double* Tout) {
    if (!ctx) return FLD_EINVAL;
    if (!E || !Tout) { ctx->err = "null pointer"; return FLD_EINVAL; }
    if (!ctx->assembled) { ctx->err = "fld_assemble first"; return FLD_ENOTREADY; }
    const int n = ctx->nx * ctx->ny;
    k_gas_update<<<grid1d(n), 256, 0, ctx->stream>>>(n, E, ctx->T, ctx->rho, ctx->kP, ctx->cv, ctx->dt, Tout);
    HIPCHK(hipGetLastError());
    return FLD_OK;
}

}  // extern "C"

namespace {

// assembly, solve and gas update without the replay guard
fld_status step_internal(fld_ctx* ctx, double* E, double* T, const double* rho, const double* kR, const double* kP,
                         const double* cv, const double* ghost, double dt, fld_solve_info* info) {
    fld_status s = fld_assemble(ctx, E, T, rho, kR, kP, cv, ghost, dt);
    if (s != FLD_OK) return s;
    s = solve_checked(ctx, E, info);
    if (s != FLD_OK) return s;
    return fld_gas_update(ctx, E, T);
}

// nsteps steps queued back to back with the kernels of fld_step, without its
// blocking synchronisations: the CG iterations run as captured two-slot
// chunks, and the host reads a chunk's solver flags (an asynchronous copy to
// one of two pinned mirrors, then its event) while the next chunk already
// runs, so the GPU never waits for the host and at most one chunk of
// early-exit slots follows convergence.  The next step is queued as soon as
// its predecessor's iterations are known to be done; records are read once
// per kStepSeg steps.
template <typename T>
fld_status steps_pipelined(fld_ctx* ctx, int32_t nsteps, double* E, double* Tg, const double* rho, const double* kR,
                           const double* kP, const double* cv, const double* ghost, double dt,
                           fld_solve_info* per_step) {
    Inner<T>& in = inner<T>(ctx);
    hipStream_t st = ctx->stream;
    const fld_options& o = ctx->opt;
    const int n = ctx->nx * ctx->ny;
    constexpr int kChunk = 2;  // even: the p buffers alternate within a chunk
    const double delta = o.precision == FLD_MIXED ? 0.01 : 1e-3;
    std::vector<fld_solve_info> h(nsteps);
    auto t0 = std::chrono::steady_clock::now();
    for (int k = 0; k < nsteps;) {
        const int m = std::min(kStepSeg, nsteps - k);
        k_zero_int<<<1, 1, 0, st>>>(ctx->seg_count);
        for (int q = 0; q < m; ++q) {
            fld_status as = enqueue_assemble(ctx, E, Tg, rho, kR, kP, cv, ghost, dt, st);
            if (as != FLD_OK) return as;
            k_init_scalars<<<1, 1, 0, st>>>(ctx->sc, o.rel_tol, delta * delta, o.inner_rtol * o.inner_rtol,
                                            o.max_inner, o.norm, o.precision == FLD_FP32 ? 0 : 1);
            enqueue_check<T>(ctx, in, E, 1, st);
            enqueue_vcycle<T>(ctx, in, st);
            // captured after the prologue's V-cycle has been queued: the chunk's
            // SpMV takes the number of r.z partials that cycle leaves
            fld_status gs = capture_chunk<T>(ctx, in, E, kChunk);
            if (gs != FLD_OK) return gs;
            // each step predicted by the one before less one iteration: the
            // relaxing sequences this serves change their counts slowly and
            // mostly downwards, and a read-ahead chunk past convergence is a
            // chunk of early-exit launches (a late read costs only the host's
            // flag-read latency)
            if (!run_chunks<T>(ctx, in, kChunk, o.max_inner, ctx->last_iters - 1, st)) {
                ctx->err = "pipelined steps: chunk launch or flag read failed";
                return FLD_EHIP;
            }
            k_correct<T><<<grid1d(n), 256, 0, st>>>(n, E, in.x, ctx->sc, 1, ctx->err_flag);
            k_gas_update<<<grid1d(n), 256, 0, st>>>(n, E, Tg, rho, kP, ctx->cv, dt, Tg);
            k_record_step<<<1, 1, 0, st>>>(ctx->sc, ctx->err_flag, ctx->seg_count, kStepSeg, (void*)ctx->seg_info,
                                           (int)ctx->h64.size());
            HIPCHK(hipGetLastError());
        }
        HIPCHK(hipStreamSynchronize(st));
        HIPCHK(hipMemcpy(h.data() + k, ctx->seg_info, sizeof(fld_solve_info) * m, hipMemcpyDeviceToHost));
        k += m;
    }
    const float ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ctx->assembled = true;
    fld_status firstbad = FLD_OK;
    for (int q = 0; q < nsteps; ++q) {
        h[q].ms = ms / nsteps;
        if (per_step) per_step[q] = h[q];
        if (h[q].status != FLD_OK && firstbad == FLD_OK) firstbad = (fld_status)h[q].status;
    }
    return firstbad;
}

}  // namespace

extern "C" {

fld_status fld_step(fld_ctx* ctx, double* E, double* T, const double* rho, const double* kR, const double* kP,
                    const double* cv, const double* ghost, double dt, fld_solve_info* info) {
    if (!ctx) return FLD_EINVAL;
    fld_status g = refuse_after_replay(ctx);
    if (g != FLD_OK) return g;
    return step_internal(ctx, E, T, rho, kR, kP, cv, ghost, dt, info);
}

fld_status fld_steps(fld_ctx* ctx, int32_t nsteps, double* E, double* T, const double* rho, const double* kR,
                     const double* kP, const double* cv, const double* ghost, double dt, fld_solve_info* per_step) {
    if (!ctx) return FLD_EINVAL;
    if (nsteps < 0) { ctx->err = "nsteps < 0"; return FLD_EINVAL; }
    fld_status g = refuse_after_replay(ctx);
    if (g != FLD_OK) return g;
    if (nsteps == 0) return FLD_OK;
    fld_status s = check_fields(ctx, E, T, rho, kR, kP, cv, ghost, dt);
    if (s != FLD_OK) return s;
    if (ctx->prof.on || !ctx->opt.use_graph) {
        // measured (events cannot be timed inside graphs) or graphs disabled:
        // fld_step calls, stopping at the first failure
        for (int k = 0; k < nsteps; ++k) {
            fld_solve_info inf{};
            fld_status sk = step_internal(ctx, E, T, rho, kR, kP, cv, ghost, dt, &inf);
            if (per_step) per_step[k] = inf;
            if (sk != FLD_OK) return sk;
        }
        return FLD_OK;
    }
    return inner_is_float(ctx) ? steps_pipelined<float>(ctx, nsteps, E, T, rho, kR, kP, cv, ghost, dt, per_step)
                               : steps_pipelined<double>(ctx, nsteps, E, T, rho, kR, kP, cv, ghost, dt, per_step);
}

fld_status fld_steps_graph(fld_ctx* ctx, int32_t nsteps, double* E, double* T, const double* rho, const double* kR,
                           const double* kP, const double* cv, const double* ghost, double dt,
                           fld_solve_info* per_step) {
    if (!ctx) return FLD_EINVAL;
    if (nsteps < 0) { ctx->err = "nsteps < 0"; return FLD_EINVAL; }
    if (nsteps == 0) return FLD_OK;
    fld_status s = check_fields(ctx, E, T, rho, kR, kP, cv, ghost, dt);
    if (s != FLD_OK) return s;
    // step 1, host-driven: measures the iteration count that sizes the budget
    fld_solve_info first{};
    fld_status s1 = step_internal(ctx, E, T, rho, kR, kP, cv, ghost, dt, &first);
    if (per_step) per_step[0] = first;
    if (s1 != FLD_OK || nsteps == 1) return s1;
    if (ctx->prof.on || !ctx->opt.use_graph) {
        // measured (events cannot be timed inside graphs) or graphs disabled
        for (int k = 1; k < nsteps; ++k) {
            fld_solve_info inf{};
            fld_status sk = step_internal(ctx, E, T, rho, kR, kP, cv, ghost, dt, &inf);
            if (per_step) per_step[k] = inf;
            if (sk != FLD_OK) return sk;
        }
        return FLD_OK;
    }
    // later steps can need well over the first step's count (c5: 85 then up
    // to 148); an unused slot costs its early-exit launches (~25, a few us
    // each), an exhausted budget a replay of the whole step
    int slots = std::min(ctx->opt.max_inner, ((first.inner_iters * 2 + 16) + 1) & ~1);
    // one captured step: assembly, hierarchy, fixed-budget solve, gas update,
    // per-step record; replayed in segments of seg steps (1, doubling after
    // every clean segment up to kStepSeg).  After each segment the host reads
    // the records once; if a step ran out of its iteration budget, the budget
    // grows by half, the step is re-captured and the segment is replayed from
    // the saved (E, T) with seg = 1 again.  Records and saved fields live in
    // the context (no allocation here).
    int seg = 1;
    if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    const int n = ctx->nx * ctx->ny;
    fld_solve_info* dinfo = ctx->seg_info;
    int* dcount = ctx->seg_count;
    double *Esave = ctx->Esave, *Tsave = ctx->Tsave;
    hipGraphExec_t ge = nullptr;
    fld_status st = FLD_OK;
    auto cleanup = [&]() {
        if (ge) (void)hipGraphExecDestroy(ge);
    };
    auto capture = [&](int budget) -> fld_status {
        if (ge) {
            (void)hipGraphExecDestroy(ge);
            ge = nullptr;
        }
        hipStream_t cs = ctx->cap_stream;
        hipGraph_t g = nullptr;
        if (join_setup(ctx, ctx->stream) != FLD_OK) return FLD_EHIP;  // no set-up left pending on the plain events
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return FLD_EHIP;
        std::swap(ctx->setup_fork, ctx->cap_fork);
        std::swap(ctx->setup_join, ctx->cap_join);
        fld_status as = enqueue_assemble(ctx, E, T, rho, kR, kP, cv, ghost, dt, cs);
        if (inner_is_float(ctx)) enqueue_solve_fixed<float>(ctx, E, budget, cs);
        else enqueue_solve_fixed<double>(ctx, E, budget, cs);
        std::swap(ctx->setup_fork, ctx->cap_fork);
        std::swap(ctx->setup_join, ctx->cap_join);
        k_gas_update<<<grid1d(n), 256, 0, cs>>>(n, E, T, rho, kP, ctx->cv, dt, T);
        k_record_step<<<1, 1, 0, cs>>>(ctx->sc, ctx->err_flag, dcount, kStepSeg, (void*)dinfo, (int)ctx->h64.size());
        hipError_t e = hipStreamEndCapture(cs, &g);
        if (as == FLD_OK && e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (as != FLD_OK) return as;
        if (e != hipSuccess) {
            ctx->err = std::string("multi-step graph: ") + hipGetErrorString(e);
            return FLD_EHIP;
        }
        return FLD_OK;
    };
    st = capture(slots);
    std::vector<fld_solve_info> h(nsteps);
    auto t0 = std::chrono::steady_clock::now();
    int k = 1;
    while (st == FLD_OK && k < nsteps) {
        const int m = std::min(seg, nsteps - k);
        const int c0 = k - 1;
        k_zero_int<<<1, 1, 0, ctx->stream>>>(dcount);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(Esave, E, sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess ||
            hipMemcpyAsync(Tsave, T, sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess) {
            st = FLD_EHIP;
            break;
        }
        ctx->replayed = true;
        for (int q = 0; q < m && st == FLD_OK; ++q)
            if (hipGraphLaunch(ge, ctx->stream) != hipSuccess) st = FLD_EHIP;
        if (st != FLD_OK || hipStreamSynchronize(ctx->stream) != hipSuccess ||
            hipMemcpy(h.data() + c0, dinfo, sizeof(fld_solve_info) * m, hipMemcpyDeviceToHost) != hipSuccess) {
            st = FLD_EHIP;
            break;
        }
        bool budget_hit = false;
        for (int q = 0; q < m; ++q)
            if (h[c0 + q].status == FLD_ENOCONV && h[c0 + q].inner_iters >= slots) budget_hit = true;
        if (budget_hit && slots < ctx->opt.max_inner) {
            slots = std::min(ctx->opt.max_inner, ((slots * 3 / 2) + 1) & ~1);
            seg = 1;
            if (hipMemcpyAsync(E, Esave, sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess ||
                hipMemcpyAsync(T, Tsave, sizeof(double) * n, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess) {
                st = FLD_EHIP;
                break;
            }
            st = capture(slots);
            continue;  // replay the segment with the larger budget
        }
        k += m;
        seg = std::min(kStepSeg, 2 * seg);
        // a relaxing sequence needs fewer iterations as it goes (the stress
        // recipe: 110 in step 2, 3 by step 100); every unused slot still costs
        // its early-exit launches (~45 launches, half of a late step's time),
        // so a budget 1.5x above what the last segment needed plus a quarter
        // (at least 4) is cut to that and re-captured; a step that overruns
        // it replays its segment with a larger budget, as above
        int need = 0;
        for (int q = 0; q < m; ++q) need = std::max(need, h[c0 + q].inner_iters);
        const int want = std::min(ctx->opt.max_inner, ((need + std::max(4, need / 4) + 2) + 1) & ~1);
        if (k < nsteps && 3 * want <= 2 * slots) {
            slots = want;
            st = capture(slots);
        }
    }
    const float ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    cleanup();
    if (st != FLD_OK) return st;
    fld_status firstbad = s1;
    for (int q = 1; q < nsteps; ++q) {
        h[q - 1].ms = ms / (nsteps - 1);
        if (per_step) per_step[q] = h[q - 1];
        if (h[q - 1].status != FLD_OK && firstbad == FLD_OK) firstbad = (fld_status)h[q - 1].status;
    }
    ctx->assembled = true;
    return firstbad;
}

fld_status fld_substep(fld_ctx* ctx, double* E, double* T, const double* rho, const double* kR, const double* kP,
                       const double* cv, const double* ghost, double dt, int32_t n_sub, double q, double dbar,
                       int32_t max_sub, double* dts, fld_solve_info* per_sub, int32_t* n_done, double* Fx,
                       double* Fy) {
    if (!ctx) return FLD_EINVAL;
    if (n_done) *n_done = 0;
    fld_status g = refuse_after_replay(ctx);
    if (g != FLD_OK) return g;
    if (max_sub < 1) { ctx->err = "max_sub must be >= 1"; return FLD_EINVAL; }
    if (!(dbar >= 0.0) || !std::isfinite(dbar)) { ctx->err = "dbar must be finite and >= 0"; return FLD_EINVAL; }
    if (dbar == 0.0 && (n_sub < 1 || n_sub > max_sub || !(q > 0.0) || !std::isfinite(q))) {
        ctx->err = "geometric sub-steps need 1 <= n_sub <= max_sub and q > 0";
        return FLD_EINVAL;
    }
    fld_status s = check_fields(ctx, E, T, rho, kR, kP, cv, ghost, dt);
    if (s != FLD_OK) return s;
    // steps 1-2 of the radiation-subsystem algorithm are taken once per step:
    // every sub-step's face coefficients and advection term come from E^n,
    // saved here, while its time derivative, C_V, beta and f use the
    // sub-step's own state and length
    const double* En = ctx->Esave;
    HIPCHK(hipMemcpyAsync(ctx->Esave, E, sizeof(double) * ctx->nx * ctx->ny, hipMemcpyDeviceToDevice, ctx->stream));
    auto sub = [&](int k, double h) -> fld_status {
        fld_solve_info inf{};
        fld_status sk = enqueue_assemble(ctx, E, T, rho, kR, kP, cv, ghost, h, ctx->stream, En);
        if (sk == FLD_OK) {
            ctx->assembled = true;
            sk = fld_solve(ctx, E, &inf);
        }
        if (sk == FLD_OK) sk = fld_gas_update(ctx, E, T);
        if (per_sub) per_sub[k] = inf;
        if (dts) dts[k] = h;
        if (n_done) *n_done = k + 1;
        if (sk == FLD_OK && (Fx || Fy)) {
            // the step's face fluxes, time-averaged over the sub-steps
            const int nf = (ctx->nx + 1) * ctx->ny + ctx->nx * (ctx->ny + 1);
            k_face_flux<<<grid1d(nf), 256, 0, ctx->stream>>>(ctx->met, ctx->We, ctx->Wn, ctx->bside, ctx->rside, E,
                                                              h, h / dt, k > 0 ? 1 : 0, Fx, Fy);
            if (hipGetLastError() != hipSuccess) return FLD_EHIP;
        }
        return sk;
    };
    if (dbar == 0.0) {
        // geometric series dt_i = dt_0 q^(i-1), dt_0 = dt (1 - q) / (1 - q^n)
        // n_sub = 1 is the step itself (the quotient would round)
        const double dt0 = n_sub == 1 ? dt : q == 1.0 ? dt / n_sub : dt * (1.0 - q) / (1.0 - std::pow(q, (double)n_sub));
        for (int k = 0; k < n_sub; ++k) {
            const fld_status sk = sub(k, (q == 1.0 || n_sub == 1) ? dt0 : dt0 * std::pow(q, (double)k));
            if (sk != FLD_OK) return sk;
        }
        return FLD_OK;
    }
    // coupling-limited: dt_k = min(remaining, min over cells dbar T C_V / |G0|)
    const int n = ctx->nx * ctx->ny;
    const int nb = grid1d(n);
    double remain = dt;
    for (int k = 0; remain > 1e-12 * dt; ++k) {
        if (k == max_sub) {
            ctx->err = "coupling-limited sub-steps exceed max_sub";
            return FLD_ENOCONV;
        }
        const double* cvk = cv;
        if (ctx->cv_p != 0.0) {
            // the sub-step's heat capacity at its start (the assembly recomputes the same)
            k_cv_law<<<nb, 256, 0, ctx->stream>>>(n, cv, T, 1.0 / ctx->cv_Tref, ctx->cv_p, ctx->cvl);
            cvk = ctx->cvl;
        }
        k_coupling_dt<<<nb, 256, 0, ctx->stream>>>(n, E, T, rho, kP, cvk, dbar, ctx->part2);
        k_reduce_min<<<1, 1024, 0, ctx->stream>>>(ctx->part2, nb, ctx->dt_lim);
        HIPCHK(hipGetLastError());
        double lim = 0.0;
        HIPCHK(hipMemcpyAsync(&lim, ctx->dt_lim, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        const double h = std::min(remain, lim);
        if (!(h > 0.0)) {
            ctx->err = "coupling-limited sub-step is not positive (T <= 0 or non-finite fields)";
            return FLD_ENONFINITE;
        }
        const fld_status sk = sub(k, h);
        if (sk != FLD_OK) return sk;
        remain -= h;
    }
    return FLD_OK;
}

fld_status fld_face_flux(fld_ctx* ctx, const double* E, double* Fx, double* Fy, double w, int32_t accumulate) {
    if (!ctx || !E) return FLD_EINVAL;
    if (!ctx->assembled) {
        ctx->err = "fld_face_flux needs an assembled step";
        return FLD_ENOTREADY;
    }
    if (!Fx && !Fy) return FLD_OK;
    const int nf = (ctx->nx + 1) * ctx->ny + ctx->nx * (ctx->ny + 1);
    k_face_flux<<<grid1d(nf), 256, 0, ctx->stream>>>(ctx->met, ctx->We, ctx->Wn, ctx->bside, ctx->rside, E, ctx->dt,
                                                      w, accumulate ? 1 : 0, Fx, Fy);
    HIPCHK(hipGetLastError());
    return FLD_OK;
}

fld_status fld_set_cv_law(fld_ctx* ctx, double T_ref, double p) {
    if (!ctx) return FLD_EINVAL;
    if (!(T_ref > 0.0) || !std::isfinite(T_ref) || !std::isfinite(p)) {
        ctx->err = "the heat-capacity law needs a finite T_ref > 0 and a finite p";
        return FLD_EINVAL;
    }
    if (p != 0.0 && !ctx->cvl && ctx->alloc(&ctx->cvl, (size_t)ctx->nx * ctx->ny) != hipSuccess) {
        ctx->err = "hipMalloc cvl";
        return FLD_ENOMEM;
    }
    ctx->cv_Tref = T_ref;
    ctx->cv_p = p;
    return FLD_OK;
}

fld_status fld_set_mass_flux(fld_ctx* ctx, const double* fx, const double* fy) {
    if (!ctx) return FLD_EINVAL;
    ctx->fx = fx;
    ctx->fy = fy;
    return FLD_OK;
}

fld_status fld_get_operator(fld_ctx* ctx, double* We, double* Wn, double* diag, double* rhs) {
    if (!ctx) return FLD_EINVAL;
    if (!ctx->assembled) { ctx->err = "fld_assemble first"; return FLD_ENOTREADY; }
    k_get_operator<<<cell_grid(ctx->nx, ctx->ny), blk2d(), 0, ctx->stream>>>(ctx->nx, ctx->ny, ctx->We, ctx->Wn, ctx->m,
                                                                             ctx->rhs, We, Wn, diag, rhs);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return FLD_OK;
}

}  // extern "C"
