// Host driver and C ABI of the batched solver (fld_batch_*, see include/fld.h).
//
// A batch is a set of independent Cartesian blocks with uniform spacing and
// ghost-cell boundaries, packed block after block.  One step of the whole
// batch is one kernel launch (one workgroup per block, largest blocks first).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "fld.h"
#include "fld_batch.hpp"

using namespace fld;

static_assert(sizeof(fld_solve_info) == sizeof(BInfo) && offsetof(fld_solve_info, rel_resid) == offsetof(BInfo, rel_resid) &&
                  offsetof(fld_solve_info, ms) == offsetof(BInfo, ms),
              "device block record must match fld_solve_info");

struct fld_batch {
    int nb = 0;
    fld_options opt{};
    hipStream_t stream = nullptr;
    std::string err;
    BCDev bc{};
    bool need_ghost = false;
    long long ncell = 0, nghost = 0, nlev = 0;
    std::vector<BBlock> hb;  // launch order
    BBlock* db = nullptr;
    std::vector<void*> allocs;
    double *We = nullptr, *Wn = nullptr, *m = nullptr, *rhs = nullptr, *s = nullptr, *r64 = nullptr;
    void *lm = nullptr, *lWe = nullptr, *lWn = nullptr, *lx = nullptr, *lb = nullptr;
    void *xi = nullptr, *p = nullptr, *q = nullptr;
    void* tr[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // transposed fine level: m, We, Wn, x, b
    BInfo* dinfo = nullptr;
    BInfo* hinfo = nullptr;
    int* dacc = nullptr;  // first non-OK status of each block over a multi-step call
    int threads = 512;
    double clock_khz = 1e5;
    size_t lds = 0;  // dynamic LDS of a launch (batch_lds of the largest level pool)

    template <typename U>
    hipError_t alloc(U** ptr, size_t count) {
        void* v = nullptr;
        hipError_t e = hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(U));
        if (e == hipSuccess) allocs.push_back(v);
        *ptr = static_cast<U*>(v);
        return e;
    }
    ~fld_batch() {
        for (void* v : allocs) (void)hipFree(v);
        if (hinfo) (void)hipHostFree(hinfo);
    }
};

namespace {

thread_local std::string t_create_err;  // reason of the last failed fld_batch_create on this thread

bool inner_float(const fld_batch* b) { return b->opt.precision != FLD_FP64; }

BOpts make_opts(const fld_options& o, double clock_khz) {
    const double delta = o.precision == FLD_MIXED ? 0.1 : 1e-3;
    BOpts r;
    r.eps = o.rel_tol;
    r.delta2 = delta * delta;
    r.inner_tol2 = o.inner_rtol * o.inner_rtol;
    r.omega = o.mg_coarse_op == FLD_MG_HALVED ? 0.5 : 1.0;
    r.clock_khz = clock_khz;
    r.max_iter = o.max_inner;
    r.norm = o.norm;
    r.reliable = o.precision == FLD_FP32 ? 0 : 1;
    r.gas = 1;
    return r;
}

// Dynamic LDS a block may use on this device (the kernel's static shared
// variables take the rest).
size_t lds_budget() {
    int dev = 0, lds = 65536;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        lds = 65536;
    return (size_t)lds - 2048;
}

template <typename T, int NT>
hipError_t set_lds() {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_batch_step<T, NT>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_budget());
}

template <typename T, int NT>
void launch_t(fld_batch* b, const BFields& f, BInfo* info, hipStream_t st) {
    BWork<T> w{b->We, b->Wn, b->m, b->rhs, b->s, b->r64,
               static_cast<T*>(b->lm), static_cast<T*>(b->lWe), static_cast<T*>(b->lWn),
               static_cast<T*>(b->lx), static_cast<T*>(b->lb),
               static_cast<T*>(b->xi), static_cast<T*>(b->p), static_cast<T*>(b->q),
               static_cast<T*>(b->tr[0]), static_cast<T*>(b->tr[1]), static_cast<T*>(b->tr[2]),
               static_cast<T*>(b->tr[3]), static_cast<T*>(b->tr[4])};
    k_batch_step<T, NT><<<b->nb, NT, b->lds, st>>>(b->db, f, w, make_opts(b->opt, b->clock_khz), info);
}

template <typename T>
void launch_p(fld_batch* b, const BFields& f, BInfo* info, hipStream_t st) {
    switch (b->threads) {
        case 256: launch_t<T, 256>(b, f, info, st); break;
        case 1024: launch_t<T, 1024>(b, f, info, st); break;
        default: launch_t<T, 512>(b, f, info, st); break;
    }
}

void launch(fld_batch* b, const BFields& f, BInfo* info, hipStream_t st) {
    if (inner_float(b)) launch_p<float>(b, f, info, st);
    else launch_p<double>(b, f, info, st);
}

fld_status check_fields(fld_batch* b, const double* E, const double* T, const double* rho, const double* kR,
                        const double* kP, const double* cv, const double* ghost, double dt) {
    if (!E || !T || !rho || !kR || !kP || !cv) { b->err = "null field pointer"; return FLD_EINVAL; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { b->err = "dt must be > 0"; return FLD_EINVAL; }
    if (b->need_ghost && !ghost) { b->err = "ghost_E required"; return FLD_EINVAL; }
    return FLD_OK;
}

BFields fields(fld_batch* b, double* E, double* T, const double* rho, const double* kR, const double* kP,
               const double* cv, const double* ghost, double dt) {
    return BFields{E, T, rho, kR, kP, cv, ghost, dt, b->opt.limiter, b->bc};
}

// Checks the options and sides of a batch (the coarsest level is clamped to
// kBCoarse cells: it is solved in the workgroup); null if they are valid.
const char* batch_options(fld_options& o, const fld_bc* bc, BCDev& bcd, bool& need_ghost) {
    if (o.precision < 0 || o.precision > 2 || o.limiter < 0 || o.limiter > 2 || o.norm < 0 || o.norm > 1 ||
        !(o.rel_tol > 0.0) || o.max_inner < 1 || !(o.inner_rtol > 0.0) || o.mg_coarse_max < 1 ||
        o.mg_coarse_max > 256 || o.mg_coarse_op < 0 || o.mg_coarse_op > 1 || o.smoother != FLD_SMOOTH_LINE)
        return "options (the batched solver uses line smoothing, mg_coarse_max in [1, 256])";
    o.mg_coarse_max = std::min(o.mg_coarse_max, kBCoarse);
    need_ghost = false;
    for (int sd = 0; sd < 4; ++sd) {
        const int k = bc ? bc[sd].kind : FLD_BC_DIRICHLET_GHOST;
        const double v = bc ? bc[sd].value : 0.0;
        if (k < 0 || k > FLD_BC_FREE_STREAM) return "boundary kind (Cartesian blocks)";
        if (k == FLD_BC_DIRICHLET_FACE && !(v > 0.0 && std::isfinite(v))) return "boundary T";
        if (k == FLD_BC_FLUX_IN && !std::isfinite(v)) return "boundary flux";
        bcd.kind[sd] = k;
        bcd.value[sd] = v;
        if (k == FLD_BC_DIRICHLET_GHOST) need_ghost = true;
    }
    return nullptr;
}

const char* block_shape(int nx, int ny, double dx, double dy) {
    if (nx < 1 || ny < 1 || nx > kBMaxSide || ny > kBMaxSide) return "block sides must be in [1, 512]";
    if (!(dx > 0.0) || !(dy > 0.0) || !std::isfinite(dx) || !std::isfinite(dy))
        return "block spacing must be finite and > 0";
    return nullptr;
}

// Multigrid levels of one block (2x2 aggregation down to mg_coarse_max cells)
// starting at packed offset lo, which advances past them; false if too many.
bool block_levels(BBlock& B, int coarse_max, long long& lo) {
    int lx = B.nx, ly = B.ny, L = 0;
    while (true) {
        if (L >= kBMaxLev) return false;
        B.lnx[L] = lx;
        B.lny[L] = ly;
        B.loff[L] = lo;
        lo += ((long long)lx * ly + 3) / 4 * 4;  // 16-byte aligned levels (vector loads)
        ++L;
        if ((long long)lx * ly <= coarse_max) break;
        lx = (lx + 1) / 2;
        ly = (ly + 1) / 2;
    }
    B.nlev = L;
    return true;
}

// LDS bytes of a block's levels from l down in the sub-cycle layout: five
// arrays per level at pitch nx + 1, the coarsest right-hand side, and one
// partial per thread of the widest workgroup (1024).
size_t sub_pool_bytes(const BBlock& B, int l, size_t ts) {
    size_t e = 0;
    for (int k = l; k < B.nlev; ++k) e += 5 * (size_t)(B.lnx[k] + 1) * B.lny[k];
    e += (size_t)B.lnx[B.nlev - 1] * B.lny[B.nlev - 1] + 1024;
    return e * ts;
}

// The finest level l >= 1 above the coarsest whose LDS pool fits `room`
// bytes (0: the block keeps every level in global memory).
int pick_sub(const BBlock& B, size_t ts, size_t room) {
    for (int l = 1; l + 1 < B.nlev; ++l)
        if (sub_pool_bytes(B, l, ts) <= room) return l;
    return 0;
}

// Dynamic LDS of the batch kernel: reductions, the coarsest inverse, and the
// union of the Gauss-Jordan workspace and the largest LDS level pool.
template <typename T>
size_t batch_lds(size_t pool) {
    using Lay = BLds<T, 512>;
    return Lay::uni + std::max(Lay::gj, pool);
}

// Metric and face arrays of one block, carved from q0 (metric_doubles(nx, ny)
// doubles): the layout k_metrics fills, then the face coordinates.
long long metric_doubles(int nx, int ny) { return 6LL * (nx + 1) + 4LL * (ny + 1) + (nx + 1) + (ny + 1); }

Metrics carve_metrics(double* q0, int X, int Y, double** xf, double** yf) {
    double *vx = q0, *ax = vx + (X + 1), *arc = ax + (X + 1), *sx = arc + (X + 1), *hxL = sx + (X + 1),
           *hxR = hxL + (X + 1);
    double *vy = hxR + (X + 1), *sy = vy + (Y + 1), *hyL = sy + (Y + 1), *hyR = hyL + (Y + 1);
    *xf = hyR + (Y + 1);
    *yf = *xf + (X + 1);
    return Metrics{X, Y, vx, vy, sx, sy, ax, hxL, hxR, hyL, hyR, arc};
}

// First non-OK status of every block, folded over the steps of one call.
__global__ void k_fold_status(const BInfo* info, int nb, int* acc) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nb && acc[k] == FLD_OK) acc[k] = info[k].status;
}

__global__ void k_zero_ints(int* p, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0;
}

fld_status first_bad(const BInfo* inf, int nb) {
    for (int k = 0; k < nb; ++k)
        if (inf[k].status != FLD_OK) return (fld_status)inf[k].status;
    return FLD_OK;
}

}  // namespace

extern "C" {

fld_status fld_batch_create(fld_batch** out, int32_t nblocks, const int32_t* nx, const int32_t* ny, const double* dx,
                            const double* dy, const fld_bc* bc, const fld_options* opt, void* stream) {
    if (!out) return FLD_EINVAL;
    *out = nullptr;
    if (nblocks < 1 || nblocks > (1 << 20) || !nx || !ny || !dx || !dy) {
        t_create_err = "nblocks must be in [1, 2^20] and the size arrays non-NULL";
        return FLD_EINVAL;
    }
    fld_batch* b = new (std::nothrow) fld_batch();
    if (!b) return FLD_ENOMEM;
    auto fail = [&](fld_status s, const char* msg) {
        t_create_err = msg;
        delete b;
        return s;
    };
    if (opt) b->opt = *opt;
    else fld_default_options(&b->opt);
    const fld_options& o = b->opt;
    if (const char* why = batch_options(b->opt, bc, b->bc, b->need_ghost)) return fail(FLD_EINVAL, why);
    b->stream = static_cast<hipStream_t>(stream);
    b->nb = nblocks;
    for (int k = 0; k < nblocks; ++k)
        if (const char* why = block_shape(nx[k], ny[k], dx[k], dy[k])) return fail(FLD_EINVAL, why);
    // layout: packed cells / ghosts in the caller's order; levels per block
    std::vector<long long> off(nblocks), goff(nblocks);
    long long nc = 0, ng = 0, nm = 0;
    for (int k = 0; k < nblocks; ++k) {
        off[k] = nc;
        goff[k] = ng;
        nc += (long long)nx[k] * ny[k];
        ng += 2LL * nx[k] + 2LL * ny[k];
        nm += metric_doubles(nx[k], ny[k]);
    }
    b->ncell = nc;
    b->nghost = ng;
    std::vector<int> order(nblocks);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return (long long)nx[a] * ny[a] > (long long)nx[c] * ny[c];
    });
    b->hb.resize(nblocks);
    long long lo = 0;
    for (int r = 0; r < nblocks; ++r) {
        const int k = order[r];
        BBlock& B = b->hb[r];
        std::memset(&B, 0, sizeof(BBlock));
        B.nx = nx[k];
        B.ny = ny[k];
        B.id = k;
        B.off = off[k];
        B.goff = goff[k];
        if (!block_levels(B, o.mg_coarse_max, lo)) return fail(FLD_EINVAL, "too many multigrid levels");
    }
    b->nlev = lo;
    {
        const size_t ts = inner_float(b) ? sizeof(float) : sizeof(double);
        const size_t uni = inner_float(b) ? BLds<float, 512>::uni : BLds<double, 512>::uni;
        const size_t budget = lds_budget();
        const size_t room = budget > uni ? budget - uni : 0;
        size_t pool = 0;
        for (BBlock& B : b->hb) {
            B.sub = pick_sub(B, ts, room);
            if (B.sub > 0) pool = std::max(pool, sub_pool_bytes(B, B.sub, ts));
        }
        b->lds = inner_float(b) ? batch_lds<float>(pool) : batch_lds<double>(pool);
    }
#define BALLOC(p, cnt) \
    if (b->alloc(&(p), (size_t)(cnt)) != hipSuccess) return fail(FLD_ENOMEM, "hipMalloc " #p)
    BALLOC(b->We, nc); BALLOC(b->Wn, nc); BALLOC(b->m, nc); BALLOC(b->rhs, nc); BALLOC(b->s, nc);
    BALLOC(b->r64, nc);
    const size_t ts = inner_float(b) ? sizeof(float) : sizeof(double);
    unsigned char *lm, *lWe, *lWn, *lx, *lbv, *xi, *pp, *qq;
    BALLOC(lm, lo * ts); BALLOC(lWe, lo * ts); BALLOC(lWn, lo * ts); BALLOC(lx, lo * ts); BALLOC(lbv, lo * ts);
    BALLOC(xi, nc * ts); BALLOC(pp, nc * ts); BALLOC(qq, nc * ts);
    b->lm = lm; b->lWe = lWe; b->lWn = lWn; b->lx = lx; b->lb = lbv; b->xi = xi; b->p = pp; b->q = qq;
    for (void*& q : b->tr) {
        unsigned char* v;
        BALLOC(v, nc * ts);
        q = v;
    }
    double* met = nullptr;
    BALLOC(met, nm);
    BALLOC(b->db, nblocks);
    BALLOC(b->dinfo, nblocks);
    BALLOC(b->dacc, nblocks);
#undef BALLOC
    if (hipHostMalloc((void**)&b->hinfo, sizeof(BInfo) * nblocks, hipHostMallocDefault) != hipSuccess)
        return fail(FLD_ENOMEM, "pinned block records");
    // metrics of every block: faces i * dx, the single-grid metric kernel
    std::vector<double> hf;
    std::vector<long long> mo(nblocks);
    {
        long long mp = 0;
        for (int k = 0; k < nblocks; ++k) {
            mo[k] = mp;
            mp += metric_doubles(nx[k], ny[k]);
        }
        hf.assign(mp, 0.0);
        for (int k = 0; k < nblocks; ++k) {
            const long long f0 = mo[k] + 6LL * (nx[k] + 1) + 4LL * (ny[k] + 1);
            for (int i = 0; i <= nx[k]; ++i) hf[f0 + i] = dx[k] * (double)i;
            for (int j = 0; j <= ny[k]; ++j) hf[f0 + nx[k] + 1 + j] = dy[k] * (double)j;
        }
    }
    if (hipMemcpy(met, hf.data(), sizeof(double) * hf.size(), hipMemcpyHostToDevice) != hipSuccess)
        return fail(FLD_EHIP, "copy faces");
    std::vector<Metrics> mets(nblocks);
    for (int k = 0; k < nblocks; ++k) {
        const int X = nx[k], Y = ny[k];
        double *xf, *yf;
        const Metrics g = carve_metrics(met + mo[k], X, Y, &xf, &yf);
        mets[k] = g;
        const int mt = std::max(X, Y) + 1;
        k_metrics<<<(mt + 255) / 256, 256, 0, b->stream>>>(0, X, Y, xf, yf, const_cast<double*>(g.vx),
                                                           const_cast<double*>(g.vy), const_cast<double*>(g.sx),
                                                           const_cast<double*>(g.sy), const_cast<double*>(g.ax),
                                                           const_cast<double*>(g.hxL), const_cast<double*>(g.hxR),
                                                           const_cast<double*>(g.hyL), const_cast<double*>(g.hyR),
                                                           const_cast<double*>(g.arc));
    }
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess)
        return fail(FLD_EHIP, "metrics kernels");
    for (auto& B : b->hb) B.met = mets[B.id];
    if (hipMemcpy(b->db, b->hb.data(), sizeof(BBlock) * nblocks, hipMemcpyHostToDevice) != hipSuccess)
        return fail(FLD_EHIP, "copy block table");
    if (hipMemset(b->xi, 0, nc * ts) != hipSuccess) return fail(FLD_EHIP, "memset");
    {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            b->clock_khz = khz;
    }
    hipError_t e;
    if (inner_float(b)) {
        e = set_lds<float, 256>();
        if (e == hipSuccess) e = set_lds<float, 512>();
        if (e == hipSuccess) e = set_lds<float, 1024>();
    } else {
        e = set_lds<double, 256>();
        if (e == hipSuccess) e = set_lds<double, 512>();
        if (e == hipSuccess) e = set_lds<double, 1024>();
    }
    if (e != hipSuccess) return fail(FLD_EHIP, "LDS size attribute");
    *out = b;
    return FLD_OK;
}

fld_status fld_batch_step(fld_batch* b, double* E, double* T, const double* rho, const double* kR, const double* kP,
                          const double* cv, const double* ghost, double dt, fld_solve_info* per_block) {
    if (!b) return FLD_EINVAL;
    fld_status s = check_fields(b, E, T, rho, kR, kP, cv, ghost, dt);
    if (s != FLD_OK) return s;
    launch(b, fields(b, E, T, rho, kR, kP, cv, ghost, dt), b->dinfo, b->stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        b->err = std::string("batch kernel: ") + hipGetErrorString(e);
        return FLD_EHIP;
    }
    if (!per_block) return FLD_OK;
    if (hipMemcpyAsync(b->hinfo, b->dinfo, sizeof(BInfo) * b->nb, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
        b->err = "batch records";
        return FLD_EHIP;
    }
    for (int k = 0; k < b->nb; ++k) std::memcpy(&per_block[k], &b->hinfo[k], sizeof(BInfo));
    return first_bad(b->hinfo, b->nb);
}

fld_status fld_batch_steps(fld_batch* b, int32_t nsteps, double* E, double* T, const double* rho, const double* kR,
                           const double* kP, const double* cv, const double* ghost, double dt,
                           fld_solve_info* per_block) {
    if (!b) return FLD_EINVAL;
    if (nsteps < 0) { b->err = "nsteps < 0"; return FLD_EINVAL; }
    if (nsteps == 0) return FLD_OK;
    fld_status s = check_fields(b, E, T, rho, kR, kP, cv, ghost, dt);
    if (s != FLD_OK) return s;
    // every step writes the block records to dinfo (the last step's remain);
    // a fold after each step keeps every block's first failure in dacc
    const BFields f = fields(b, E, T, rho, kR, kP, cv, ghost, dt);
    const int fg = (b->nb + 255) / 256;
    auto queue = [&](hipStream_t st) {
        k_zero_ints<<<fg, 256, 0, st>>>(b->dacc, b->nb);
        for (int k = 0; k < nsteps; ++k) {
            launch(b, f, b->dinfo, st);
            k_fold_status<<<fg, 256, 0, st>>>(b->dinfo, b->nb, b->dacc);
        }
    };
    fld_status st = FLD_OK;
    if (b->opt.use_graph) {
        // the nsteps kernel nodes (and their folds) form one graph
        hipStream_t cs = nullptr;
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            queue(cs);
            e = hipStreamEndCapture(cs, &g);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipGraphLaunch(ge, b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
        if (ge) (void)hipGraphExecDestroy(ge);
        if (g) (void)hipGraphDestroy(g);
        if (cs) (void)hipStreamDestroy(cs);
        if (e != hipSuccess) {
            b->err = std::string("batch graph: ") + hipGetErrorString(e);
            st = FLD_EHIP;
        }
    } else {
        queue(b->stream);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(b->stream) != hipSuccess) {
            b->err = "batch kernels";
            st = FLD_EHIP;
        }
    }
    if (st != FLD_OK) return st;
    std::vector<int> acc(b->nb);
    if (hipMemcpy(acc.data(), b->dacc, sizeof(int) * b->nb, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(b->hinfo, b->dinfo, sizeof(BInfo) * b->nb, hipMemcpyDeviceToHost) != hipSuccess) {
        b->err = "batch records";
        return FLD_EHIP;
    }
    // the first failing block in the caller's order, as a single batch step reports it
    for (int k = 0; k < b->nb && st == FLD_OK; ++k) st = (fld_status)acc[k];
    if (per_block)
        for (int k = 0; k < b->nb; ++k) std::memcpy(&per_block[k], &b->hinfo[k], sizeof(BInfo));
    return st;
}

fld_status fld_batch_set_threads(fld_batch* b, int32_t threads) {
    if (!b) return FLD_EINVAL;
    if (threads != 256 && threads != 512 && threads != 1024) {
        b->err = "threads must be 256, 512 or 1024";
        return FLD_EINVAL;
    }
    b->threads = threads;
    return FLD_OK;
}

fld_status fld_batch_get_threads(const fld_batch* b, int32_t* threads) {
    if (!b || !threads) return FLD_EINVAL;
    *threads = b->threads;
    return FLD_OK;
}

fld_status fld_batch_sizes(const fld_batch* b, int64_t* cells, int64_t* ghosts) {
    if (!b) return FLD_EINVAL;
    if (cells) *cells = b->ncell;
    if (ghosts) *ghosts = b->nghost;
    return FLD_OK;
}

const char* fld_batch_last_error(const fld_batch* b) { return b ? b->err.c_str() : t_create_err.c_str(); }

void fld_batch_destroy(fld_batch* b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    delete b;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// fld_block_step_noalloc: one block stepped by the batch kernel with every
// byte of its device workspace in a static per-device array.
// ---------------------------------------------------------------------------

namespace {

constexpr size_t kScratchBytes = size_t(4) << 20;  // 4 MiB per device
constexpr int kMaxDevices = 64;

// The workspace.  In host code this name is only a stand-in for the symbol:
// kernels and copies use the address from hipGetSymbolAddress (scratch_ptr).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
double g_clock_khz[kMaxDevices] = {};

constexpr size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// Device address of this device's scratch array, the batch kernel's LDS
// attribute and the wall-clock rate, set up once per device (the caller's
// current device); null on failure.
void* scratch_for_current_device(double* clock_khz) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        if (set_lds<float, 512>() != hipSuccess || set_lds<double, 512>() != hipSuccess) return nullptr;
        int khz = 0;
        g_clock_khz[dev] =
            (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0) ? khz : 1e5;
        g_scratch_ptr[dev] = ptr;
    }
    *clock_khz = g_clock_khz[dev];
    return g_scratch_ptr[dev];
}

__global__ void k_put_block(BBlock blk, BBlock* dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = blk;
}

__global__ void k_block_faces(double* xf, int nx, double dx, double* yf, int ny, double dy) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t <= nx) xf[t] = dx * (double)t;
    if (t <= ny) yf[t] = dy * (double)t;
}

}  // namespace

extern "C" {

fld_status fld_block_step_noalloc(int32_t nx, int32_t ny, double dx, double dy, const fld_bc* bc,
                                  const fld_options* opt, double* E, double* T, const double* rho, const double* kR,
                                  const double* kP, const double* cv, const double* ghost, double dt, void* stream,
                                  fld_solve_info* info) {
    fld_options o;
    if (opt) o = *opt;
    else fld_default_options(&o);
    BCDev bcd{};
    bool need_ghost = false;
    if (const char* why = batch_options(o, bc, bcd, need_ghost)) { t_create_err = why; return FLD_EINVAL; }
    if (const char* why = block_shape(nx, ny, dx, dy)) { t_create_err = why; return FLD_EINVAL; }
    if (!E || !T || !rho || !kR || !kP || !cv) { t_create_err = "null field pointer"; return FLD_EINVAL; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { t_create_err = "dt must be > 0"; return FLD_EINVAL; }
    if (need_ghost && !ghost) { t_create_err = "ghost_E required"; return FLD_EINVAL; }
    // the block's table entry and levels, and the scratch layout (256-byte pieces)
    BBlock B;
    std::memset(&B, 0, sizeof(BBlock));
    B.nx = nx;
    B.ny = ny;
    long long lo = 0;
    if (!block_levels(B, o.mg_coarse_max, lo)) { t_create_err = "too many multigrid levels"; return FLD_EINVAL; }
    const size_t n = (size_t)nx * ny;
    const size_t ts = o.precision != FLD_FP64 ? sizeof(float) : sizeof(double);
    const size_t uni = ts == sizeof(float) ? BLds<float, 512>::uni : BLds<double, 512>::uni;
    {
        const size_t budget = lds_budget();
        B.sub = pick_sub(B, ts, budget > uni ? budget - uni : 0);
    }
    const size_t pool = B.sub > 0 ? sub_pool_bytes(B, B.sub, ts) : 0;
    const size_t lds = ts == sizeof(float) ? batch_lds<float>(pool) : batch_lds<double>(pool);
    const size_t nm = (size_t)metric_doubles(nx, ny);
    const size_t need = align256(sizeof(BBlock)) + align256(sizeof(BInfo)) + align256(nm * sizeof(double)) +
                        6 * align256(n * sizeof(double)) + 5 * align256((size_t)lo * ts) + 8 * align256(n * ts);
    if (need > kScratchBytes) {
        t_create_err = "block needs " + std::to_string(need) + " bytes of workspace; the static workspace holds " +
                       std::to_string(kScratchBytes);
        return FLD_EINVAL;
    }
    double clock_khz = 1e5;
    unsigned char* base = static_cast<unsigned char*>(scratch_for_current_device(&clock_khz));
    if (!base) { t_create_err = "static workspace: hipGetSymbolAddress or kernel attribute failed"; return FLD_EHIP; }
    size_t at = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base + at;
        at += align256(bytes);
        return p;
    };
    BBlock* db = reinterpret_cast<BBlock*>(take(sizeof(BBlock)));
    BInfo* dinfo = reinterpret_cast<BInfo*>(take(sizeof(BInfo)));
    double *xf, *yf;
    B.met = carve_metrics(reinterpret_cast<double*>(take(nm * sizeof(double))), nx, ny, &xf, &yf);
    double* w64[6];
    for (auto& q : w64) q = reinterpret_cast<double*>(take(n * sizeof(double)));
    void* lv[5];
    for (auto& q : lv) q = take((size_t)lo * ts);
    void* vec[8];  // xi, p, q, then the transposed fine level
    for (auto& q : vec) q = take(n * ts);
    // set-up kernels: table entry, faces at i dx and j dy, metrics (no copies from the host)
    hipStream_t st = static_cast<hipStream_t>(stream);
    const Metrics& g = B.met;
    const int mt = std::max(nx, ny) + 1;
    k_put_block<<<1, 1, 0, st>>>(B, db);
    k_block_faces<<<(mt + 255) / 256, 256, 0, st>>>(xf, nx, dx, yf, ny, dy);
    k_metrics<<<(mt + 255) / 256, 256, 0, st>>>(0, nx, ny, xf, yf, const_cast<double*>(g.vx), const_cast<double*>(g.vy),
                                                const_cast<double*>(g.sx), const_cast<double*>(g.sy),
                                                const_cast<double*>(g.ax), const_cast<double*>(g.hxL),
                                                const_cast<double*>(g.hxR), const_cast<double*>(g.hyL),
                                                const_cast<double*>(g.hyR), const_cast<double*>(g.arc));
    const BFields f{E, T, rho, kR, kP, cv, ghost, dt, o.limiter, bcd};
    const BOpts bo = make_opts(o, clock_khz);
    if (ts == sizeof(float)) {
        BWork<float> w{w64[0], w64[1], w64[2], w64[3], w64[4], w64[5],
                       static_cast<float*>(lv[0]), static_cast<float*>(lv[1]), static_cast<float*>(lv[2]),
                       static_cast<float*>(lv[3]), static_cast<float*>(lv[4]),
                       static_cast<float*>(vec[0]), static_cast<float*>(vec[1]), static_cast<float*>(vec[2]),
                       static_cast<float*>(vec[3]), static_cast<float*>(vec[4]), static_cast<float*>(vec[5]),
                       static_cast<float*>(vec[6]), static_cast<float*>(vec[7])};
        k_batch_step<float, 512><<<1, 512, lds, st>>>(db, f, w, bo, dinfo);
    } else {
        BWork<double> w{w64[0], w64[1], w64[2], w64[3], w64[4], w64[5],
                        static_cast<double*>(lv[0]), static_cast<double*>(lv[1]), static_cast<double*>(lv[2]),
                        static_cast<double*>(lv[3]), static_cast<double*>(lv[4]),
                        static_cast<double*>(vec[0]), static_cast<double*>(vec[1]), static_cast<double*>(vec[2]),
                        static_cast<double*>(vec[3]), static_cast<double*>(vec[4]), static_cast<double*>(vec[5]),
                        static_cast<double*>(vec[6]), static_cast<double*>(vec[7])};
        k_batch_step<double, 512><<<1, 512, lds, st>>>(db, f, w, bo, dinfo);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        t_create_err = std::string("block kernel: ") + hipGetErrorString(e);
        return FLD_EHIP;
    }
    if (!info) return FLD_OK;
    BInfo h{};
    if (hipMemcpyAsync(&h, dinfo, sizeof(BInfo), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        t_create_err = "block record";
        return FLD_EHIP;
    }
    std::memcpy(info, &h, sizeof(BInfo));
    return (fld_status)h.status;
}

}  // extern "C"
