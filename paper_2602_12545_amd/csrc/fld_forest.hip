// Multilevel FLD radiation step on a statically refined block forest, solved
// as one matrix across the refinement levels (Section 3.2.2: a coarse cell
// at a level jump couples directly to both fine cells of that side, each
// through the fine face's own D; Section 4: the solver needs only the
// neighbour lists precomputed from the grid hierarchy).
//
// Layout: leaf cells numbered block after block, each block row-major.  The
// host builds once, at create, the interior faces (two cells, area, the two
// centre-to-face normal distances) and the domain-boundary faces, and for
// every cell an ELL list of up to eight (face, neighbour) slots, stored
// slot-major so that a wavefront reads consecutive entries.  A step is:
// one thread per face for the conductances (the uniform grid's face
// function), one thread per cell for the boundary and cell terms (the T
// elimination of the single grid), then Jacobi-preconditioned CG in FP64 with
// matrix-free gather products m x + sum W (x - x_nb), per-workgroup partial
// sums reduced in a fixed order by one workgroup, and the device-side
// control of the single-grid solver (iterations queued in captured chunks
// that exit at once when the solve is done).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "fld.h"
#include "fld_kernels.hpp"

using namespace fld;

namespace {

constexpr int kFT = 256;          // threads per workgroup of the cell and face kernels
constexpr int kFMaxWG = 2048;     // grid cap (partial sums per reduction)
constexpr int kFRed = 1024;       // threads of the reducing workgroup
constexpr int kFSlots = 8;        // neighbour slots per cell (two per side at a level jump)
constexpr int kFChunk = 16;       // CG iterations per captured chunk (even: p buffers alternate)

struct FScal {
    double rz, alpha, beta, rel, rel_row, rel_sc, den_row, den_sc, eps;
    int iter, max_iter, done, status, norm;
};

inline int grid_for(long long n) { return (int)std::max<long long>(1, std::min<long long>((n + kFT - 1) / kFT, kFMaxWG)); }

// Sums of NV partials per workgroup (stored [k][nwg]) by one workgroup, in a
// fixed order; results in out[0..NV).
template <int NV>
__device__ inline void reduce_parts(const double* part, int nwg, double* out) {
    __shared__ double sh[kFRed / 64];
    for (int k = 0; k < NV; ++k) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nwg; b += kFRed) v += part[(size_t)k * nwg + b];
        const double s = block_sum(v, sh);
        if (threadIdx.x == 0) out[k] = s;
    }
}

__global__ __launch_bounds__(kFT) void k_ff_faces(int nf, const int* __restrict__ fa, const int* __restrict__ fb,
                                                  const double* __restrict__ area, const double* __restrict__ ha,
                                                  const double* __restrict__ hb, const double* __restrict__ E,
                                                  const double* __restrict__ rho, const double* __restrict__ kR,
                                                  double dt, int lim, double* __restrict__ W) {
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += gridDim.x * blockDim.x) {
        const int a = fa[f], b = fb[f];
        W[f] = face_W(E[a], kR[a] * rho[a], E[b], kR[b] * rho[b], ha[f], hb[f], area[f], dt, lim);
    }
}

struct FCellIn {
    const double *E, *T, *rho, *kR, *kP, *cv;
    double dt;
    int lim;
    BCDev bc;
};

// Cell terms (T eliminated, Section 3.2.1 coefficient list): mass
// m = dV (1 + beta f) + boundary diagonal, 1 / diag, right-hand side.
__global__ __launch_bounds__(kFT) void k_ff_cells(int n, const double* __restrict__ dV, const int* __restrict__ ellf,
                                                  const int* __restrict__ bslot, const int* __restrict__ bside,
                                                  const double* __restrict__ barea, const double* __restrict__ bh,
                                                  const double* __restrict__ W, FCellIn in, double* __restrict__ m,
                                                  double* __restrict__ dinv, double* __restrict__ rhs,
                                                  double* __restrict__ bd, double* __restrict__ br, int* err) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const double E = in.E[c], T = in.T[c], rho = in.rho[c], kR = in.kR[c], kP = in.kP[c], cv = in.cv[c];
        const bool ok = isfinite(E) && E > 0.0 && isfinite(T) && T > 0.0 && isfinite(rho) && rho > 0.0 &&
                        isfinite(kR) && kR > 0.0 && isfinite(kP) && kP >= 0.0 && isfinite(cv) && cv >= 0.0;
        if (!ok) atomicOr(err, 1);
        const double sig = kR * rho;
        double bdc = 0.0, brc = 0.0;
        for (int s = 0; s < 2; ++s) {
            const int f = bslot[(size_t)s * n + c];
            if (f < 0) continue;
            const int sd = bside[f];
            double d = 0.0, r = 0.0;
            boundary_face(in.bc.kind[sd], in.bc.value[sd], 0.0, E, sig, bh[f], barea[f], in.dt, in.lim, d, r);
            bd[f] = d;
            br[f] = r;
            bdc += d;
            brc += r;
        }
        double sumW = 0.0;
        for (int s = 0; s < kFSlots; ++s) {
            const int f = ellf[(size_t)s * n + c];
            if (f >= 0) sumW += W[f];
        }
        const double CV = rho * cv;
        const double beta = kP * rho * kC * in.dt;
        const double T3 = T * T * T;
        const double X = 4.0 * beta * kARad * T3;
        const double den = CV + X;
        const double fr = den > 0.0 ? CV / den : 1.0;
        const double vol = dV[c];
        const double mass = vol * (1.0 + beta * fr);
        m[c] = mass + bdc;
        dinv[c] = 1.0 / ((mass + sumW) + bdc);
        rhs[c] = vol * (E + beta * fr * kARad * T3 * T) + brc;
    }
}

// A x in flux form, m x + sum over the cell's faces of W (x - x_nb).
__device__ inline double apply_row(int c, int n, double xc, const double* __restrict__ m, const double* __restrict__ W,
                                   const int* __restrict__ ellf, const int* __restrict__ elln,
                                   const double* __restrict__ x) {
    double acc = m[c] * xc;
    for (int s = 0; s < kFSlots; ++s) {
        const int f = ellf[(size_t)s * n + c];
        if (f >= 0) acc += W[f] * (xc - x[elln[(size_t)s * n + c]]);
    }
    return acc;
}

// r = rhs - A x, z = D^-1 r; the old search direction is cleared (a new CG
// start); partials: r.z, |r / dV|^2, |rhs / dV|^2, rhs.D^-1.rhs.
__global__ __launch_bounds__(kFT) void k_ff_init(int n, const double* __restrict__ x, const double* __restrict__ rhs,
                                                 const double* __restrict__ m, const double* __restrict__ dinv,
                                                 const double* __restrict__ W, const int* __restrict__ ellf,
                                                 const int* __restrict__ elln, const double* __restrict__ dV,
                                                 double* __restrict__ r, double* __restrict__ z,
                                                 double* __restrict__ p0, double* __restrict__ part) {
    __shared__ double sh[kFT / 64];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const double b = rhs[c];
        const double rc = b - apply_row(c, n, x[c], m, W, ellf, elln, x);
        const double zc = dinv[c] * rc;
        r[c] = rc;
        z[c] = zc;
        p0[c] = 0.0;
        const double iv = 1.0 / dV[c];
        a0 += rc * zc;
        a1 += (rc * iv) * (rc * iv);
        a2 += (b * iv) * (b * iv);
        a3 += b * dinv[c] * b;
    }
    const int nwg = gridDim.x;
    double s;
    s = block_sum(a0, sh); if (threadIdx.x == 0) part[0 * nwg + blockIdx.x] = s;
    s = block_sum(a1, sh); if (threadIdx.x == 0) part[1 * nwg + blockIdx.x] = s;
    s = block_sum(a2, sh); if (threadIdx.x == 0) part[2 * nwg + blockIdx.x] = s;
    s = block_sum(a3, sh); if (threadIdx.x == 0) part[3 * nwg + blockIdx.x] = s;
}

__global__ __launch_bounds__(kFRed) void k_ff_init_reduce(const double* part, int nwg, FScal* sc) {
    __shared__ double v[4];
    reduce_parts<4>(part, nwg, v);
    if (threadIdx.x == 0) {
        sc->rz = v[0];
        sc->den_row = v[2];
        sc->den_sc = v[3];
        sc->rel_row = v[2] > 0.0 ? sqrt(v[1] / v[2]) : 0.0;
        sc->rel_sc = v[3] > 0.0 ? sqrt(fmax(v[0], 0.0) / v[3]) : 0.0;
        sc->rel = sc->norm == 0 ? sc->rel_row : sc->rel_sc;
        sc->beta = 0.0;
        sc->done = (sc->rel <= sc->eps || !(v[0] > 0.0)) ? 1 : 0;
        if (!isfinite(v[0]) || !isfinite(v[1])) {
            sc->status = ST_ENONFINITE;
            sc->done = 1;
        }
    }
}

// p_new = z + beta p_old (also recomputed for the neighbours from their z and
// p_old, so that no workgroup reads what another writes), q = A p_new; p.q partials.
__global__ __launch_bounds__(kFT) void k_ff_spmv(int n, const double* __restrict__ z, const double* __restrict__ p_old,
                                                 double* __restrict__ p_new, double* __restrict__ q,
                                                 const double* __restrict__ m, const double* __restrict__ W,
                                                 const int* __restrict__ ellf, const int* __restrict__ elln,
                                                 const FScal* sc, double* __restrict__ part) {
    if (sc->done) return;
    __shared__ double sh[kFT / 64];
    const double beta = sc->beta;
    double a = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const double pc = z[c] + beta * p_old[c];
        double acc = m[c] * pc;
        for (int s = 0; s < kFSlots; ++s) {
            const int f = ellf[(size_t)s * n + c];
            if (f >= 0) {
                const int k = elln[(size_t)s * n + c];
                acc += W[f] * (pc - (z[k] + beta * p_old[k]));
            }
        }
        p_new[c] = pc;
        q[c] = acc;
        a += pc * acc;
    }
    const double s = block_sum(a, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kFRed) void k_ff_alpha(const double* part, int nwg, FScal* sc) {
    if (sc->done) return;
    __shared__ double v[1];
    reduce_parts<1>(part, nwg, v);
    if (threadIdx.x == 0) {
        const double pq = v[0];
        if (!(pq > 0.0) || !isfinite(pq)) {
            sc->status = ST_EBREAKDOWN;
            sc->done = 1;
        } else {
            sc->alpha = sc->rz / pq;
        }
    }
}

__global__ __launch_bounds__(kFT) void k_ff_update(int n, double* __restrict__ x, double* __restrict__ r,
                                                   double* __restrict__ z, const double* __restrict__ p,
                                                   const double* __restrict__ q, const double* __restrict__ dinv,
                                                   const double* __restrict__ dV, const FScal* sc,
                                                   double* __restrict__ part) {
    if (sc->done) return;
    __shared__ double sh[kFT / 64];
    const double al = sc->alpha;
    double a0 = 0.0, a1 = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        x[c] += al * p[c];
        const double rc = r[c] - al * q[c];
        const double zc = dinv[c] * rc;
        r[c] = rc;
        z[c] = zc;
        const double iv = 1.0 / dV[c];
        a0 += rc * zc;
        a1 += (rc * iv) * (rc * iv);
    }
    const int nwg = gridDim.x;
    double s = block_sum(a0, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    s = block_sum(a1, sh);
    if (threadIdx.x == 0) part[nwg + blockIdx.x] = s;
}

__global__ __launch_bounds__(kFRed) void k_ff_beta(const double* part, int nwg, FScal* sc) {
    if (sc->done) return;
    __shared__ double v[2];
    reduce_parts<2>(part, nwg, v);
    if (threadIdx.x == 0) {
        const double rz = v[0];
        sc->beta = rz / sc->rz;
        sc->rz = rz;
        sc->iter += 1;
        sc->rel_row = sc->den_row > 0.0 ? sqrt(v[1] / sc->den_row) : 0.0;
        sc->rel_sc = sc->den_sc > 0.0 ? sqrt(fmax(rz, 0.0) / sc->den_sc) : 0.0;
        sc->rel = sc->norm == 0 ? sc->rel_row : sc->rel_sc;
        if (!isfinite(rz)) {
            sc->status = ST_EBREAKDOWN;
            sc->done = 1;
        } else if (sc->rel <= sc->eps) {
            sc->done = 1;
        } else if (sc->iter >= sc->max_iter) {
            sc->status = ST_ENOCONV;
            sc->done = 1;
        }
    }
}

__global__ void k_ff_scalars(FScal* sc, double eps, int max_iter, int norm, int* err) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        FScal v;
        v.rz = v.alpha = v.beta = v.rel = v.rel_row = v.rel_sc = v.den_row = v.den_sc = 0.0;
        v.eps = eps;
        v.iter = 0;
        v.max_iter = max_iter;
        v.done = 0;
        v.status = ST_OK;
        v.norm = norm;
        *sc = v;
        *err = 0;
    }
}

inline uint64_t cell_key(int L, long long i, long long j) {
    return ((uint64_t)L << 58) | ((uint64_t)i << 29) | (uint64_t)j;
}

}  // namespace

struct fld_forest {
    int n = 0, nf = 0, nb = 0;
    fld_options opt{};
    BCDev bc{};
    hipStream_t stream = nullptr, cap = nullptr;
    std::string err;
    std::vector<void*> allocs;
    std::vector<int> hlevel;
    std::vector<double> hxc, hyc;
    // geometry
    double *dV = nullptr, *farea = nullptr, *fha = nullptr, *fhb = nullptr, *barea = nullptr, *bh = nullptr;
    int *fa = nullptr, *fb = nullptr, *ellf = nullptr, *elln = nullptr, *bslot = nullptr, *bside = nullptr;
    // operator and solver state
    double *W = nullptr, *m = nullptr, *dinv = nullptr, *rhs = nullptr, *bd = nullptr, *br = nullptr;
    double *x = nullptr, *r = nullptr, *z = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr, *part = nullptr;
    FScal* sc = nullptr;
    FScal* hsc = nullptr;
    int* errf = nullptr;
    int* herr = nullptr;
    int grid = 1;
    hipGraphExec_t chunk = nullptr;

    template <typename U>
    hipError_t alloc(U** p, size_t cnt) {
        void* v = nullptr;
        hipError_t e = hipMalloc(&v, std::max<size_t>(cnt, 1) * sizeof(U));
        if (e == hipSuccess) allocs.push_back(v);
        *p = static_cast<U*>(v);
        return e;
    }
    ~fld_forest() {
        if (chunk) (void)hipGraphExecDestroy(chunk);
        if (stream) (void)hipStreamSynchronize(stream);
        for (void* v : allocs) (void)hipFree(v);
        if (hsc) (void)hipHostFree(hsc);
        if (herr) (void)hipHostFree(herr);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

thread_local std::string t_forest_err;

void enqueue_iterations(fld_forest* F, int count, hipStream_t st) {
    const int n = F->n, g = F->grid;
    for (int k = 0; k < count; ++k) {
        double* po = (k & 1) ? F->p1 : F->p0;
        double* pn = (k & 1) ? F->p0 : F->p1;
        k_ff_spmv<<<g, kFT, 0, st>>>(n, F->z, po, pn, F->q, F->m, F->W, F->ellf, F->elln, F->sc, F->part);
        k_ff_alpha<<<1, kFRed, 0, st>>>(F->part, g, F->sc);
        k_ff_update<<<g, kFT, 0, st>>>(n, F->x, F->r, F->z, pn, F->q, F->dinv, F->dV, F->sc, F->part);
        k_ff_beta<<<1, kFRed, 0, st>>>(F->part, g, F->sc);
    }
}

fld_status read_scalars(fld_forest* F) {
    if (hipMemcpyAsync(F->hsc, F->sc, sizeof(FScal), hipMemcpyDeviceToHost, F->stream) != hipSuccess ||
        hipStreamSynchronize(F->stream) != hipSuccess) {
        F->err = "reading the solver state";
        return FLD_EHIP;
    }
    return FLD_OK;
}

}  // namespace

extern "C" {

fld_status fld_forest_create(fld_forest** out, int32_t nblocks, const fld_forest_block* blocks, int32_t nx0,
                             int32_t ny0, double dx0, double dy0, const fld_bc* bc, const fld_options* opt,
                             void* stream) {
    if (!out) return FLD_EINVAL;
    *out = nullptr;
    auto bad = [&](const std::string& msg) {
        t_forest_err = msg;
        return FLD_EINVAL;
    };
    if (nblocks < 1 || !blocks || nx0 < 1 || ny0 < 1 || !(dx0 > 0.0) || !(dy0 > 0.0) || !std::isfinite(dx0) ||
        !std::isfinite(dy0))
        return bad("need blocks, a level-0 domain of nx0 x ny0 >= 1 cells and spacings > 0");
    fld_options o;
    if (opt) o = *opt;
    else fld_default_options(&o);
    if (o.precision != FLD_FP64) return bad("the forest solver runs in FP64 (precision = FLD_FP64)");
    if (o.limiter < 0 || o.limiter > 2 || o.norm < 0 || o.norm > 1 || !(o.rel_tol > 0.0) || o.max_inner < 1)
        return bad("options");
    BCDev bcd{};
    for (int sd = 0; sd < 4; ++sd) {
        const int k = bc ? bc[sd].kind : FLD_BC_REFLECT;
        const double v = bc ? bc[sd].value : 0.0;
        if (k != FLD_BC_REFLECT && k != FLD_BC_DIRICHLET_FACE && k != FLD_BC_FLUX_IN && k != FLD_BC_FREE_STREAM)
            return bad("forest sides: reflecting, Dirichlet face, fixed inward flux or free streaming");
        if (k == FLD_BC_DIRICHLET_FACE && !(v > 0.0 && std::isfinite(v))) return bad("boundary temperature");
        if (k == FLD_BC_FLUX_IN && !std::isfinite(v)) return bad("boundary flux");
        bcd.kind[sd] = k;
        bcd.value[sd] = v;
    }
    // leaf cells, block after block, each block row-major
    std::unordered_map<uint64_t, int> cell;
    std::vector<int> lev, ci, cj;
    long long total = 0;
    int Lmax = 0;
    for (int b = 0; b < nblocks; ++b) {
        const fld_forest_block& B = blocks[b];
        if (B.level < 0 || B.level > 16 || B.nx < 1 || B.ny < 1 || B.i0 < 0 || B.j0 < 0)
            return bad("block " + std::to_string(b) + ": level in [0, 16], sizes >= 1, origin >= 0");
        const long long NXL = (long long)nx0 << B.level, NYL = (long long)ny0 << B.level;
        if (B.i0 + (long long)B.nx > NXL || B.j0 + (long long)B.ny > NYL)
            return bad("block " + std::to_string(b) + " extends beyond the domain");
        total += (long long)B.nx * B.ny;
        if (total > (1LL << 27)) return bad("more than 2^27 cells");
        Lmax = std::max(Lmax, (int)B.level);
        for (int j = B.j0; j < B.j0 + B.ny; ++j)
            for (int i = B.i0; i < B.i0 + B.nx; ++i) {
                if (!cell.emplace(cell_key(B.level, i, j), (int)lev.size()).second)
                    return bad("block " + std::to_string(b) + " overlaps another block");
                lev.push_back(B.level);
                ci.push_back(i);
                cj.push_back(j);
            }
    }
    const int n = (int)lev.size();
    // exact cover: no leaf inside another leaf, and the areas add up
    long double area = 0.0L;
    for (int c = 0; c < n; ++c) {
        for (int k = 1; k <= lev[c]; ++k)
            if (cell.count(cell_key(lev[c] - k, ci[c] >> k, cj[c] >> k)))
                return bad("a refined cell lies inside a leaf cell of a coarser block");
        area += std::ldexp(1.0L, -2 * lev[c]);
    }
    if (std::fabs((double)(area - (long double)nx0 * ny0)) > 1e-9 * nx0 * ny0)
        return bad("the blocks do not cover the domain");
    // faces
    std::vector<int> fa, fb, bcell, bsd;
    std::vector<double> farea, fha, fhb, barea, bhh;
    std::vector<std::vector<std::pair<int, int>>> slots(n);  // (face, neighbour)
    std::vector<std::vector<int>> bsl(n);
    const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
    for (int c = 0; c < n; ++c) {
        const int L = lev[c];
        const double hx = dx0 / (double)(1LL << L), hy = dy0 / (double)(1LL << L);
        const long long NXL = (long long)nx0 << L, NYL = (long long)ny0 << L;
        for (int sd = 0; sd < 4; ++sd) {
            const int axis = sd < 2 ? 0 : 1;
            const long long ii = ci[c] + di[sd], jj = cj[c] + dj[sd];
            const double ar = axis == 0 ? hy : hx, hh = 0.5 * (axis == 0 ? hx : hy);
            if (ii < 0 || jj < 0 || ii >= NXL || jj >= NYL) {
                bsl[c].push_back((int)bcell.size());
                bcell.push_back(c);
                bsd.push_back(sd);
                barea.push_back(ar);
                bhh.push_back(hh);
                continue;
            }
            auto s = cell.find(cell_key(L, ii, jj));
            if (s != cell.end()) {
                if (sd == 1 || sd == 3) {  // each same-level face once, from its lower cell
                    const int f = (int)fa.size();
                    fa.push_back(c);
                    fb.push_back(s->second);
                    farea.push_back(ar);
                    fha.push_back(hh);
                    fhb.push_back(hh);
                    slots[c].push_back({f, s->second});
                    slots[s->second].push_back({f, c});
                }
                continue;
            }
            auto co = L > 0 ? cell.find(cell_key(L - 1, ii >> 1, jj >> 1)) : cell.end();
            if (co != cell.end()) {
                // level jump seen from the fine cell: one fine face to the coarse cell
                const int k = co->second;
                const double hc = 0.5 * (axis == 0 ? 2.0 * hx : 2.0 * hy);
                const bool lower_is_coarse = (sd == 0 || sd == 2);
                const int f = (int)fa.size();
                fa.push_back(lower_is_coarse ? k : c);
                fb.push_back(lower_is_coarse ? c : k);
                farea.push_back(ar);
                fha.push_back(lower_is_coarse ? hc : hh);
                fhb.push_back(lower_is_coarse ? hh : hc);
                slots[c].push_back({f, k});
                slots[k].push_back({f, c});
                continue;
            }
            // finer neighbours add their faces themselves; one of them must exist
            const long long fi = axis == 0 ? 2 * ii + (di[sd] < 0 ? 1 : 0) : 2 * ii;
            const long long fj = axis == 1 ? 2 * jj + (dj[sd] < 0 ? 1 : 0) : 2 * jj;
            if (!cell.count(cell_key(L + 1, fi, fj)))
                return bad("cell " + std::to_string(c) + " has no neighbour on side " + std::to_string(sd) +
                           ": the forest is not 2:1 balanced");
        }
    }
    for (int c = 0; c < n; ++c)
        if ((int)slots[c].size() > kFSlots) return bad("more than eight neighbours (not 2:1 balanced)");
    fld_forest* F = new (std::nothrow) fld_forest();
    if (!F) return FLD_ENOMEM;
    auto fail = [&](fld_status s, const std::string& msg) {
        t_forest_err = msg;
        delete F;
        return s;
    };
    F->n = n;
    F->nf = (int)fa.size();
    F->nb = (int)bcell.size();
    F->opt = o;
    F->bc = bcd;
    F->stream = static_cast<hipStream_t>(stream);
    F->grid = grid_for(n);
    F->hlevel = lev;
    F->hxc.resize(n);
    F->hyc.resize(n);
    std::vector<double> hdV(n);
    for (int c = 0; c < n; ++c) {
        const double hx = dx0 / (double)(1LL << lev[c]), hy = dy0 / (double)(1LL << lev[c]);
        F->hxc[c] = (ci[c] + 0.5) * hx;
        F->hyc[c] = (cj[c] + 0.5) * hy;
        hdV[c] = hx * hy;
    }
    std::vector<int> hellf((size_t)kFSlots * n, -1), helln((size_t)kFSlots * n, 0), hbs((size_t)2 * n, -1);
    for (int c = 0; c < n; ++c) {
        for (size_t s = 0; s < slots[c].size(); ++s) {
            hellf[s * n + c] = slots[c][s].first;
            helln[s * n + c] = slots[c][s].second;
        }
        for (size_t s = 0; s < bsl[c].size(); ++s) hbs[s * n + c] = bsl[c][s];
    }
    const size_t nn = n, nf = std::max(F->nf, 1), nb = std::max(F->nb, 1);
#define FALLOC(p, cnt) \
    if (F->alloc(&(p), (cnt)) != hipSuccess) return fail(FLD_ENOMEM, "hipMalloc " #p)
    FALLOC(F->dV, nn); FALLOC(F->farea, nf); FALLOC(F->fha, nf); FALLOC(F->fhb, nf); FALLOC(F->barea, nb);
    FALLOC(F->bh, nb); FALLOC(F->fa, nf); FALLOC(F->fb, nf); FALLOC(F->ellf, kFSlots * nn);
    FALLOC(F->elln, kFSlots * nn); FALLOC(F->bslot, 2 * nn); FALLOC(F->bside, nb);
    FALLOC(F->W, nf); FALLOC(F->m, nn); FALLOC(F->dinv, nn); FALLOC(F->rhs, nn); FALLOC(F->bd, nb); FALLOC(F->br, nb);
    FALLOC(F->x, nn); FALLOC(F->r, nn); FALLOC(F->z, nn); FALLOC(F->p0, nn); FALLOC(F->p1, nn); FALLOC(F->q, nn);
    FALLOC(F->part, 4 * (size_t)kFMaxWG); FALLOC(F->sc, 1); FALLOC(F->errf, 1);
#undef FALLOC
    if (hipHostMalloc((void**)&F->hsc, sizeof(FScal), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&F->herr, sizeof(int), hipHostMallocDefault) != hipSuccess)
        return fail(FLD_ENOMEM, "pinned scalars");
    auto up = [&](void* d, const void* h, size_t bytes) {
        return bytes == 0 || hipMemcpy(d, h, bytes, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (!up(F->dV, hdV.data(), sizeof(double) * n) || !up(F->farea, farea.data(), sizeof(double) * F->nf) ||
        !up(F->fha, fha.data(), sizeof(double) * F->nf) || !up(F->fhb, fhb.data(), sizeof(double) * F->nf) ||
        !up(F->barea, barea.data(), sizeof(double) * F->nb) || !up(F->bh, bhh.data(), sizeof(double) * F->nb) ||
        !up(F->fa, fa.data(), sizeof(int) * F->nf) || !up(F->fb, fb.data(), sizeof(int) * F->nf) ||
        !up(F->ellf, hellf.data(), sizeof(int) * hellf.size()) ||
        !up(F->elln, helln.data(), sizeof(int) * helln.size()) ||
        !up(F->bslot, hbs.data(), sizeof(int) * hbs.size()) || !up(F->bside, bsd.data(), sizeof(int) * F->nb))
        return fail(FLD_EHIP, "copy of the forest tables");
    if (hipStreamCreateWithFlags(&F->cap, hipStreamNonBlocking) != hipSuccess) return fail(FLD_EHIP, "capture stream");
    *out = F;
    return FLD_OK;
}

fld_status fld_forest_sizes(const fld_forest* F, int64_t* cells, int64_t* faces, int64_t* boundary_faces) {
    if (!F) return FLD_EINVAL;
    if (cells) *cells = F->n;
    if (faces) *faces = F->nf;
    if (boundary_faces) *boundary_faces = F->nb;
    return FLD_OK;
}

fld_status fld_forest_cells(const fld_forest* F, double* xc, double* yc, int32_t* level) {
    if (!F) return FLD_EINVAL;
    for (int c = 0; c < F->n; ++c) {
        if (xc) xc[c] = F->hxc[c];
        if (yc) yc[c] = F->hyc[c];
        if (level) level[c] = F->hlevel[c];
    }
    return FLD_OK;
}

fld_status fld_forest_step(fld_forest* F, double* E, double* T, const double* rho, const double* kR, const double* kP,
                           const double* cv, double dt, fld_solve_info* info) {
    if (!F) return FLD_EINVAL;
    if (!E || !T || !rho || !kR || !kP || !cv) { F->err = "null field pointer"; return FLD_EINVAL; }
    if (!(dt > 0.0) || !std::isfinite(dt)) { F->err = "dt must be > 0"; return FLD_EINVAL; }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = F->stream;
    const int n = F->n, g = F->grid;
    const fld_options& o = F->opt;
    k_ff_scalars<<<1, 1, 0, st>>>(F->sc, o.rel_tol, o.max_inner, o.norm, F->errf);
    if (F->nf > 0)
        k_ff_faces<<<grid_for(F->nf), kFT, 0, st>>>(F->nf, F->fa, F->fb, F->farea, F->fha, F->fhb, E, rho, kR, dt,
                                                    o.limiter, F->W);
    const FCellIn in{E, T, rho, kR, kP, cv, dt, o.limiter, F->bc};
    k_ff_cells<<<g, kFT, 0, st>>>(n, F->dV, F->ellf, F->bslot, F->bside, F->barea, F->bh, F->W, in, F->m, F->dinv,
                                  F->rhs, F->bd, F->br, F->errf);
    if (hipMemcpyAsync(F->x, E, sizeof(double) * n, hipMemcpyDeviceToDevice, st) != hipSuccess) {
        F->err = "copy of E";
        return FLD_EHIP;
    }
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(F->herr, F->errf, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess) {
        F->err = "assembly kernels";
        return FLD_EHIP;
    }
    if (!F->chunk) {
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamBeginCapture(F->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            enqueue_iterations(F, kFChunk, F->cap);
            e = hipStreamEndCapture(F->cap, &gr);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&F->chunk, gr, nullptr, nullptr, 0);
        if (gr) (void)hipGraphDestroy(gr);
        if (e != hipSuccess) {
            F->err = std::string("CG chunk graph: ") + hipGetErrorString(e);
            return FLD_EHIP;
        }
    }
    // CG from E^n; after the recurrence converges, the true residual decides
    // (a restart from the current iterate if it has drifted above the target)
    int restarts = 0;
    fld_status s = FLD_OK;
    while (true) {
        k_ff_init<<<g, kFT, 0, st>>>(n, F->x, F->rhs, F->m, F->dinv, F->W, F->ellf, F->elln, F->dV, F->r, F->z, F->p0,
                                     F->part);
        k_ff_init_reduce<<<1, kFRed, 0, st>>>(F->part, g, F->sc);
        if ((s = read_scalars(F)) != FLD_OK) return s;
        if (*F->herr) { F->err = "non-finite or out-of-domain field values"; s = FLD_ENONFINITE; break; }
        if (F->hsc->status != ST_OK) { s = (fld_status)F->hsc->status; break; }
        if (F->hsc->rel <= o.rel_tol) break;
        if (F->hsc->iter >= o.max_inner || restarts > 8) { s = FLD_ENOCONV; break; }
        ++restarts;
        while (true) {
            if (hipGraphLaunch(F->chunk, st) != hipSuccess) { F->err = "chunk launch"; return FLD_EHIP; }
            if ((s = read_scalars(F)) != FLD_OK) return s;
            if (F->hsc->done) break;
        }
        if (F->hsc->status == ST_EBREAKDOWN || F->hsc->status == ST_ENONFINITE) { s = (fld_status)F->hsc->status; break; }
        if (F->hsc->status == ST_ENOCONV) {
            // budget spent: evaluate the true residual once more and stop
            k_ff_init<<<g, kFT, 0, st>>>(n, F->x, F->rhs, F->m, F->dinv, F->W, F->ellf, F->elln, F->dV, F->r, F->z,
                                         F->p0, F->part);
            k_ff_init_reduce<<<1, kFRed, 0, st>>>(F->part, g, F->sc);
            if ((s = read_scalars(F)) != FLD_OK) return s;
            s = F->hsc->rel <= o.rel_tol ? FLD_OK : FLD_ENOCONV;
            break;
        }
    }
    const FScal h = *F->hsc;
    if (s == FLD_OK) {
        k_gas_update<<<g, 256, 0, st>>>(n, F->x, T, rho, kP, cv, dt, T);
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(E, F->x, sizeof(double) * n, hipMemcpyDeviceToDevice, st) != hipSuccess) {
            F->err = "gas update";
            return FLD_EHIP;
        }
    } else {
        (void)hipMemcpyAsync(E, F->x, sizeof(double) * n, hipMemcpyDeviceToDevice, st);
        if (F->err.empty()) F->err = fld_status_string(s);
    }
    if (info) {
        (void)hipStreamSynchronize(st);
        info->status = s;
        info->outer_iters = restarts;
        info->inner_iters = h.iter;
        info->mg_levels = 0;
        info->rel_resid = o.norm == 0 ? h.rel_row : h.rel_sc;
        info->rel_resid_row = h.rel_row;
        info->rel_resid_scaled = h.rel_sc;
        info->ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return s;
}

const char* fld_forest_last_error(const fld_forest* F) { return F ? F->err.c_str() : t_forest_err.c_str(); }

void fld_forest_destroy(fld_forest* F) { delete F; }

}  // extern "C"
