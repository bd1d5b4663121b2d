// Batched implicit radiation step for many independent blocks (static mesh
// refinement blocks in their independent form, Section 3.2.2: every block sees
// its neighbours and parent only through ghost values).
//
// One workgroup owns one block for a whole step: assembly (FP64), the
// multigrid hierarchy, the reliable-update MG-preconditioned CG solve and the
// gas update, with workgroup barriers as the only synchronisation.  Blocks of
// 16 .. 128 cells per side keep their working set in L2 / Infinity Cache, and
// the coarsest-level inverse and all scalars stay on chip; one launch covers
// every block of the batch.
#pragma once

#include "fld_kernels.hpp"
#include "fld_line.hpp"
#include "fld_sub.hpp"

namespace fld {

constexpr int kBMaxLev = 12;       // multigrid levels per block
constexpr int kBCoarse = 64;       // coarsest level: at most this many cells, inverted densely
constexpr int kBLineL = 8;         // cells per thread chunk in the line solves
constexpr int kBMaxSide = 64 * kBLineL;  // block side limit: a line fits one wavefront
constexpr int kBRedDoubles = 128;  // reduction scratch (5 sums x 16 waves)

struct BBlock {
    int nx, ny, nlev, id;          // id: index of the block in the caller's order
    int sub;                       // first level held in LDS for the whole step (0: none)
    long long off, goff;           // first cell / first ghost value in the packed arrays
    long long loff[kBMaxLev];      // first cell of each level in the packed level arrays
    int lnx[kBMaxLev], lny[kBMaxLev];
    Metrics met;
};

struct BFields {
    double* E;
    double* T;
    const double *rho, *kR, *kP, *cv, *ghost;
    double dt;
    int lim;
    BCDev bc;
};

template <typename T>
struct BWork {
    double *We, *Wn, *m, *rhs, *s, *r64;  // FP64 operator and true residual (packed cells)
    T *lm, *lWe, *lWn, *lx, *lb;          // inner-precision hierarchy, all levels (packed)
    T *xi, *p, *q;                        // inner CG vectors of the fine level (packed cells)
    T *mT, *WeT, *WnT, *xT, *bT;          // the fine level transposed (columns as rows), packed cells
};

struct BOpts {
    double eps, delta2, inner_tol2, omega;
    double clock_khz;  // rate of the device wall clock (per-block timing)
    int max_iter, norm, reliable, gas;
};

// Layout of fld_solve_info.
struct BInfo {
    int32_t status, outer_iters, inner_iters, mg_levels;
    double rel_resid, rel_resid_row, rel_resid_scaled;
    float ms;
};

template <typename T, int NT>
struct BLds {
    static constexpr size_t red = 0;
    static constexpr size_t ainv = kBRedDoubles * sizeof(double);
    // transpose tile: th rows of tc, pitch tc + 1 (16.6 KB in either precision)
    static constexpr int th = sizeof(T) == 4 ? 64 : 32, tc = 64;
    static constexpr size_t tile = ainv + (size_t)kBCoarse * kBCoarse * sizeof(T);
    static constexpr size_t uni = tile + (size_t)th * (tc + 1) * sizeof(T);
    static constexpr size_t gj = sizeof(double) * ((size_t)kBCoarse * kBCoarse + kBCoarse);
    static constexpr size_t bytes = uni + gj;
};

// Workgroup sums / maximum, the result in every thread (fixed order: deterministic).
template <int NT, int NV>
__device__ inline void wg_sum(double (&v)[NV], double* red) {
    constexpr int NW = NT / 64;
#pragma unroll
    for (int q = 0; q < NV; ++q)
        for (int o = 32; o > 0; o >>= 1) v[q] += __shfl_xor(v[q], o, 64);
    const int t = threadIdx.x;
    if ((t & 63) == 0)
#pragma unroll
        for (int q = 0; q < NV; ++q) red[q * NW + (t >> 6)] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += red[q * NW + w];
        v[q] = s;
    }
    __syncthreads();
}

template <int NT>
__device__ inline double wg_max(double v, double* red) {
    constexpr int NW = NT / 64;
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int t = threadIdx.x;
    if ((t & 63) == 0) red[t >> 6] = v;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < NW; ++w) r = fmax(r, red[w]);
    __syncthreads();
    return r;
}

// Loop over the n cells of a block, U cells per thread per round: the loads
// of all U cells (ld) are issued before any result is stored (st), so U
// memory round trips overlap.  Per thread, cells are visited in increasing
// order (t, t + NT, ...), which keeps partial sums in a fixed order.
template <int NT, int U, class Ld, class St>
__device__ inline void cells(int n, Ld ld, St st) {
    using S = decltype(ld(0));
    for (int c0 = threadIdx.x; c0 < n; c0 += NT * U) {
        S v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int c = c0 + k * NT;
            if (c < n) v[k] = ld(c);
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const int c = c0 + k * NT;
            if (c < n) st(c, v[k]);
        }
    }
}

template <typename T>
struct V2 {
    T a, b;
};
template <typename T>
struct V4 {
    T a, b, c, d;
};

// One zebra half-sweep of a level of one block (dir 0: rows, 1: columns),
// lines spread over the workgroup's wavefronts, then a barrier.  Not inlined:
// the kernel runs one copy of the sweep code for every level and direction,
// which keeps it resident in the instruction cache.
template <typename T, int NT>
__device__ __attribute__((noinline)) void b_sweep(int nx, int ny, int dir, int par, int zero, const T* m,
                                                  const T* We, const T* Wn, const T* b, T* x) {
    const int na = dir ? ny : nx, nl = dir ? nx : ny;
    const long long sa = dir ? nx : 1, sl = dir ? 1 : nx;
    const T* Wa = dir ? Wn : We;
    const T* Wc = dir ? We : Wn;
    constexpr bool BF = sizeof(T) == 8;  // branch-free loads pay off in binary64 only (measured)
    if (zero)
        wave_line_sweep<T, kBLineL, true, BF, true>(na, nl, par, sa, sl, m, Wa, Wc, b, x, threadIdx.x >> 6, NT / 64);
    else
        wave_line_sweep<T, kBLineL, false, BF, true>(na, nl, par, sa, sl, m, Wa, Wc, b, x, threadIdx.x >> 6, NT / 64);
    __syncthreads();
}

// Residual b - A x (flux form) of a level summed over 2x2 aggregates: the
// right-hand side of the next coarser level.  One coarse cell per thread, the
// loads of its (up to) four fine cells issued together.
template <typename T, int NT>
__device__ __attribute__((noinline)) void b_restrict(int nx, int ny, const T* __restrict__ m, const T* __restrict__ We,
                           const T* __restrict__ Wn, const T* __restrict__ b, const T* __restrict__ x,
                           T* __restrict__ bc, int nxc, int nyc) {
    struct Q {
        T v[4][11];  // per fine cell: x, x_e, x_w, x_n, x_s, W_e, W_w, W_n, W_s, m, b
    };
    cells<NT, (sizeof(T) == 4 ? 2 : 1)>(
        nxc * nyc,
        [&](int C) {
            Q q;
            const int I = C % nxc, J = C / nxc;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int i = 2 * I + (a & 1), j = 2 * J + (a >> 1);
                const bool ok = i < nx && j < ny;
                const long long c = (long long)j * nx + i;
                T* v = q.v[a];
                v[0] = ok ? x[c] : T(0);
                v[1] = (ok && i + 1 < nx) ? x[c + 1] : T(0);
                v[2] = (ok && i > 0) ? x[c - 1] : T(0);
                v[3] = (ok && j + 1 < ny) ? x[c + nx] : T(0);
                v[4] = (ok && j > 0) ? x[c - nx] : T(0);
                v[5] = ok ? We[c] : T(0);
                v[6] = (ok && i > 0) ? We[c - 1] : T(0);
                v[7] = ok ? Wn[c] : T(0);
                v[8] = (ok && j > 0) ? Wn[c - nx] : T(0);
                v[9] = ok ? m[c] : T(0);
                v[10] = ok ? b[c] : T(0);
            }
            return q;
        },
        [&](int C, const Q& q) {
            const int I = C % nxc, J = C / nxc;
            T sum = T(0);
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const int i = 2 * I + (a & 1), j = 2 * J + (a >> 1);
                if (i >= nx || j >= ny) continue;
                const T* v = q.v[a];
                const T xc = v[0];
                T fl = T(0);
                if (i + 1 < nx) fl += v[5] * (xc - v[1]);
                if (i > 0) fl += v[6] * (xc - v[2]);
                if (j + 1 < ny) fl += v[7] * (xc - v[3]);
                if (j > 0) fl += v[8] * (xc - v[4]);
                sum += v[10] - v[9] * xc - fl;
            }
            bc[C] = sum;
        });
}

// 2x2 aggregation: masses summed, the conductances crossing between two
// aggregates summed and scaled by omega.
template <typename T, int NT>
__device__ void b_coarsen(int nx, int ny, const T* __restrict__ m, const T* __restrict__ We, const T* __restrict__ Wn,
                          int nxc, int nyc, T* __restrict__ mc, T* __restrict__ Wec, T* __restrict__ Wnc, T omega) {
    for (int C = threadIdx.x; C < nxc * nyc; C += NT) {
        const int I = C % nxc, J = C / nxc;
        T ms = T(0), e = T(0), nn = T(0);
        for (int bj = 0; bj < 2; ++bj) {
            const int j = 2 * J + bj;
            if (j >= ny) continue;
            for (int a = 0; a < 2; ++a) {
                const int i = 2 * I + a;
                if (i < nx) ms += m[(long long)j * nx + i];
            }
            if (2 * I + 2 < nx) e += We[(long long)j * nx + 2 * I + 1];
        }
        if (2 * J + 2 < ny)
            for (int a = 0; a < 2; ++a) {
                const int i = 2 * I + a;
                if (i < nx) nn += Wn[(long long)(2 * J + 1) * nx + i];
            }
        mc[C] = ms;
        Wec[C] = omega * e;
        Wnc[C] = omega * nn;
    }
}

// Dense inverse of the coarsest level (Gauss-Jordan in FP64, the matrix is SPD
// and diagonally dominant: no pivoting), stored in the inner precision in LDS.
template <typename T, int NT>
__device__ void b_coarse_setup(int nx, int ny, const T* __restrict__ m, const T* __restrict__ We,
                               const T* __restrict__ Wn, double* A, double* col, T* ainv) {
    const int n = nx * ny, t = threadIdx.x;
    for (int q = t; q < n * n; q += NT) A[q] = 0.0;
    __syncthreads();
    for (int c = t; c < n; c += NT) {
        const int i = c % nx, j = c / nx;
        const double e = (i + 1 < nx) ? (double)We[c] : 0.0;
        const double w = (i > 0) ? (double)We[c - 1] : 0.0;
        const double no = (j + 1 < ny) ? (double)Wn[c] : 0.0;
        const double so = (j > 0) ? (double)Wn[c - nx] : 0.0;
        A[c * n + c] = (double)m[c] + ((w + e) + (so + no));
        if (i + 1 < nx) A[c * n + c + 1] = -e;
        if (i > 0) A[c * n + c - 1] = -w;
        if (j + 1 < ny) A[c * n + c + nx] = -no;
        if (j > 0) A[c * n + c - nx] = -so;
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double p = A[k * n + k];
        for (int i = t; i < n; i += NT) col[i] = A[i * n + k];
        __syncthreads();
        for (int i = t; i < n; i += NT) A[i * n + k] = (i == k) ? 1.0 : 0.0;
        __syncthreads();
        for (int jj = t; jj < n; jj += NT) A[k * n + jj] /= p;
        __syncthreads();
        for (int q = t; q < n * n; q += NT) {
            const int i = q / n, jj = q % n;
            if (i != k) A[q] -= col[i] * A[k * n + jj];
        }
        __syncthreads();
    }
    for (int q = t; q < n * n; q += NT) ainv[q] = (T)A[q];
    __syncthreads();
}

template <typename T, int NT>
__device__ __attribute__((noinline)) void b_coarse_solve(int n, const T* ainv, const T* __restrict__ b, T* __restrict__ x) {
    for (int c = threadIdx.x; c < n; c += NT) {
        T s = T(0);
        for (int k = 0; k < n; ++k) s += ainv[c * n + k] * b[k];
        x[c] = s;
    }
    __syncthreads();
}

// dst = src transposed: src is ny rows of nx, dst nx rows of ny.  The block
// goes through LDS in tiles of TH rows x TC columns (row pitch TC + 1, so the
// column reads hit distinct banks), read along src rows and written along dst
// rows; each thread holds TH TC / NT elements of a tile, and the next tile's
// loads are issued before the current tile is written out.
template <typename T, int NT, int TH, int TC>
__device__ __attribute__((noinline)) void b_transpose(int nx, int ny, const T* __restrict__ src, T* __restrict__ dst,
                                                      T* tile) {
    constexpr int PER = TH * TC / NT;
    static_assert(PER >= 1 && PER * NT == TH * TC, "tile must split evenly over the workgroup");
    const int t = threadIdx.x;
    const int ntx = (nx + TC - 1) / TC, nt = ntx * ((ny + TH - 1) / TH);
    T v[PER];
    auto load = [&](int k) {
        const int j0 = (k / ntx) * TH, i0 = (k % ntx) * TC;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int e = t + p * NT, r = e / TC, c = e % TC;
            v[p] = (j0 + r < ny && i0 + c < nx) ? src[(long long)(j0 + r) * nx + i0 + c] : T(0);
        }
    };
    load(0);
    for (int k = 0; k < nt; ++k) {
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int e = t + p * NT;
            tile[(e / TC) * (TC + 1) + e % TC] = v[p];
        }
        __syncthreads();
        if (k + 1 < nt) load(k + 1);
        const int j0 = (k / ntx) * TH, i0 = (k % ntx) * TC;
#pragma unroll
        for (int p = 0; p < PER; ++p) {
            const int e = t + p * NT, c = e / TH, r = e % TH;
            if (j0 + r < ny && i0 + c < nx) dst[(long long)(i0 + c) * ny + j0 + r] = tile[r * (TC + 1) + c];
        }
        __syncthreads();
    }
}

// The LDS levels' V-cycle as a function of its own (not inlined into
// b_vcycle: each keeps its own register budget).
template <typename T, int NT>
__device__ __attribute__((noinline)) void b_sub_vcycle(const SubCycle<T>& S, T* pool) {
    sub_vcycle<T, NT>(S, pool);
}

// z = V(r): one V-cycle from a zero start; r is the fine level's b array and z
// its x array.  Pre-smoothing on the launched levels: rows (even, odd), then
// columns (even, odd), except on the fine level, which runs its columns first
// (from the zero start) as row sweeps of its transposed copy (strided column
// loads cost about twice the rows' time on one CU), then its rows.  The coarse
// correction (piecewise constant) is added, then post-smoothing runs in the
// reverse order, so the preconditioner is symmetric.  The fine level takes
// four transposes per cycle: b and x into the column layout, x back twice.
template <typename T, int NT>
__device__ __attribute__((noinline)) void b_vcycle(const BBlock& B, BWork<T> w, const T* ainv,
                                                   const SubCycle<T>* S, T* pool, T* tile) {
    using Lay = BLds<T, NT>;
    const int Lv = B.nlev;
    const long long bo = B.off;  // the block's fine-level cells in the packed transposed arrays
    T* xT = w.xT + bo;
    T* bT = w.bT + bo;
    if (Lv == 1) {
        const long long o = B.loff[0];
        b_coarse_solve<T, NT>(B.lnx[0] * B.lny[0], ainv, w.lb + o, w.lx + o);
        return;
    }
    // levels from Ls down run in LDS (S), or only the coarsest is solved
    const int Ls = S ? B.sub : Lv - 1;
    for (int l = 0; l < Ls; ++l) {
        const int nx = B.lnx[l], ny = B.lny[l];
        const long long o = B.loff[l], oc = B.loff[l + 1];
        const T *m = w.lm + o, *We = w.lWe + o, *Wn = w.lWn + o, *b = w.lb + o;
        T* x = w.lx + o;
        if (l == 0) {
            b_transpose<T, NT, Lay::th, Lay::tc>(nx, ny, b, bT, tile);
            b_sweep<T, NT>(ny, nx, 0, 0, 1, w.mT + bo, w.WeT + bo, w.WnT + bo, bT, xT);
            b_sweep<T, NT>(ny, nx, 0, 1, 0, w.mT + bo, w.WeT + bo, w.WnT + bo, bT, xT);
            b_transpose<T, NT, Lay::th, Lay::tc>(ny, nx, xT, x, tile);
            b_sweep<T, NT>(nx, ny, 0, 0, 0, m, We, Wn, b, x);
            b_sweep<T, NT>(nx, ny, 0, 1, 0, m, We, Wn, b, x);
        } else {
            b_sweep<T, NT>(nx, ny, 0, 0, 1, m, We, Wn, b, x);
            b_sweep<T, NT>(nx, ny, 0, 1, 0, m, We, Wn, b, x);
            b_sweep<T, NT>(nx, ny, 1, 0, 0, m, We, Wn, b, x);
            b_sweep<T, NT>(nx, ny, 1, 1, 0, m, We, Wn, b, x);
        }
        b_restrict<T, NT>(nx, ny, m, We, Wn, b, x, w.lb + oc, B.lnx[l + 1], B.lny[l + 1]);
        __syncthreads();
    }
    if (S) {
        // the restricted residual into the LDS level, its V-cycle there, and
        // the correction back for the prolongation above
        const SubLevel<T>& L0 = S->lv[0];
        const int nx = L0.nx, n = nx * L0.ny;
        const long long o = B.loff[Ls];
        T* pb = pool + L0.off + 3 * L0.size;
        for (int c = threadIdx.x; c < n; c += NT) pb[(c / nx) * L0.pitch + c % nx] = w.lb[o + c];
        __syncthreads();
        b_sub_vcycle<T, NT>(*S, pool);
        const T* px = pool + L0.off + 4 * L0.size;
        for (int c = threadIdx.x; c < n; c += NT) w.lx[o + c] = px[(c / nx) * L0.pitch + c % nx];
        __syncthreads();
    } else {
        const long long o = B.loff[Lv - 1];
        b_coarse_solve<T, NT>(B.lnx[Lv - 1] * B.lny[Lv - 1], ainv, w.lb + o, w.lx + o);
    }
    for (int l = Ls - 1; l >= 0; --l) {
        const int nx = B.lnx[l], ny = B.lny[l], nxc = B.lnx[l + 1];
        const long long o = B.loff[l], oc = B.loff[l + 1];
        const T *m = w.lm + o, *We = w.lWe + o, *Wn = w.lWn + o, *b = w.lb + o;
        T* x = w.lx + o;
        const T* ec = w.lx + oc;
        cells<NT, 8>(
            nx * ny,
            [&](int c) {
                const int i = c % nx, j = c / nx;
                return V2<T>{x[c], ec[(long long)(j >> 1) * nxc + (i >> 1)]};
            },
            [&](int c, const V2<T>& v) { x[c] = v.a + v.b; });
        __syncthreads();
        if (l == 0) {
            b_sweep<T, NT>(nx, ny, 0, 1, 0, m, We, Wn, b, x);
            b_sweep<T, NT>(nx, ny, 0, 0, 0, m, We, Wn, b, x);
            b_transpose<T, NT, Lay::th, Lay::tc>(nx, ny, x, xT, tile);
            b_sweep<T, NT>(ny, nx, 0, 1, 0, w.mT + bo, w.WeT + bo, w.WnT + bo, bT, xT);
            b_sweep<T, NT>(ny, nx, 0, 0, 0, w.mT + bo, w.WeT + bo, w.WnT + bo, bT, xT);
            b_transpose<T, NT, Lay::th, Lay::tc>(ny, nx, xT, x, tile);
        } else {
            b_sweep<T, NT>(nx, ny, 1, 1, 0, m, We, Wn, b, x);
            b_sweep<T, NT>(nx, ny, 1, 0, 0, m, We, Wn, b, x);
            b_sweep<T, NT>(nx, ny, 0, 1, 0, m, We, Wn, b, x);
            b_sweep<T, NT>(nx, ny, 0, 0, 0, m, We, Wn, b, x);
        }
    }
}

// One implicit step of every block: blockIdx.x selects the block (the table
// is ordered by decreasing size so the largest blocks start first).
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_batch_step(const BBlock* __restrict__ blocks, BFields f, BWork<T> w, BOpts o,
                                                   BInfo* __restrict__ info) {
    extern __shared__ __align__(16) unsigned char b_smem[];
    __shared__ int s_err;
    using Lay = BLds<T, NT>;
    double* red = reinterpret_cast<double*>(b_smem + Lay::red);
    T* ainv = reinterpret_cast<T*>(b_smem + Lay::ainv);
    T* tile = reinterpret_cast<T*>(b_smem + Lay::tile);
    double* gjA = reinterpret_cast<double*>(b_smem + Lay::uni);
    double* gjc = gjA + kBCoarse * kBCoarse;

    const long long t_start = wall_clock64();
    const BBlock& B = blocks[blockIdx.x];
    const int nx = B.nx, ny = B.ny, n = nx * ny, t = threadIdx.x;
    const long long off = B.off;
    double* E = f.E + off;
    double* Tg = f.T + off;
    double *We64 = w.We + off, *Wn64 = w.Wn + off, *m64 = w.m + off, *rhs = w.rhs + off, *s64 = w.s + off;
    double* r64 = w.r64 + off;
    const Metrics& g = B.met;

    // ---- assembly (FP64) and the block's normalisation mu = max diagonal
    if (t == 0) s_err = 0;
    __syncthreads();
    double mu;
    {
        AsmIn ain{E, Tg, f.rho + off, f.kR + off, f.kP + off, f.cv + off, f.ghost ? f.ghost + B.goff : nullptr,
                  f.dt, f.lim, f.bc};
        AsmOut aout{We64, Wn64, m64, rhs, s64, &s_err, nullptr};
        double dmax = 0.0;
        for (int c = t; c < n; c += NT) dmax = fmax(dmax, assemble_cell(g, ain, aout, c % nx, c / nx));
        mu = wg_max<NT>(dmax, red);  // same value in every thread; s_err is final after its barriers
    }
    const int err = s_err;
    int status = ST_OK, iter = 0, nchecks = 0;
    double rel_row = 0.0, rel_sc = 0.0, rel_sel = 0.0;
    if (err) {
        status = ST_ENONFINITE;
    } else {
        // ---- hierarchy: fine level / mu in the inner precision, aggregation, coarse inverse
        const double smu = 1.0 / mu;
        {
            const long long o0 = B.loff[0];
            for (int c = t; c < n; c += NT) {
                w.lm[o0 + c] = (T)(m64[c] * smu);
                w.lWe[o0 + c] = (T)(We64[c] * smu);
                w.lWn[o0 + c] = (T)(Wn64[c] * smu);
                w.xi[off + c] = T(0);
            }
            __syncthreads();
            // the transposed fine level: rows are the columns, the couplings
            // along them the north ones, across them the east ones
            b_transpose<T, NT, Lay::th, Lay::tc>(nx, ny, w.lm + o0, w.mT + off, tile);
            b_transpose<T, NT, Lay::th, Lay::tc>(nx, ny, w.lWn + o0, w.WeT + off, tile);
            b_transpose<T, NT, Lay::th, Lay::tc>(nx, ny, w.lWe + o0, w.WnT + off, tile);
            for (int l = 0; l + 1 < B.nlev; ++l) {
                const long long a = B.loff[l], c = B.loff[l + 1];
                b_coarsen<T, NT>(B.lnx[l], B.lny[l], w.lm + a, w.lWe + a, w.lWn + a, B.lnx[l + 1], B.lny[l + 1],
                                 w.lm + c, w.lWe + c, w.lWn + c, (T)o.omega);
                __syncthreads();
            }
            const long long cl = B.loff[B.nlev - 1];
            b_coarse_setup<T, NT>(B.lnx[B.nlev - 1], B.lny[B.nlev - 1], w.lm + cl, w.lWe + cl, w.lWn + cl, gjA, gjc,
                                  ainv);
        }
        // levels from B.sub down stay in LDS for the whole step, laid out as
        // the single grid's sub-cycle lays them out (five arrays per level at
        // pitch nx + 1, the coarsest right-hand side, one partial per
        // thread); the pool overlays the Gauss-Jordan workspace, free now
        __shared__ SubCycle<T> s_sub;
        T* pool = reinterpret_cast<T*>(b_smem + Lay::uni);
        const SubCycle<T>* S = nullptr;
        if (B.sub > 0) {
            if (t == 0) {
                SubCycle<T>& Q = s_sub;
                Q.nlev = B.nlev - B.sub;
                int po = 0;
                for (int k = 0; k < Q.nlev; ++k) {
                    const int l = B.sub + k;
                    const int pitch = B.lnx[l] + 1;
                    Q.lv[k] = SubLevel<T>{B.lnx[l], B.lny[l], w.lm + B.loff[l], w.lWe + B.loff[l], w.lWn + B.loff[l],
                                          po, 0, pitch, pitch * B.lny[l]};
                    po += 5 * pitch * B.lny[l];
                }
                Q.Ainv = ainv;
                Q.bc_off = po;
                Q.part_off = po + B.lnx[B.nlev - 1] * B.lny[B.nlev - 1];
                Q.kcyc = 0;
                Q.k_off = Q.part_off + NT;
            }
            __syncthreads();
            for (int k = 0; k + 1 < s_sub.nlev; ++k) {
                const SubLevel<T>& L = s_sub.lv[k];
                T* pm = pool + L.off;
                for (int c = t; c < L.nx * L.ny; c += NT) {
                    const int cl = (c / L.nx) * L.pitch + c % L.nx;
                    pm[cl] = L.m[c];
                    pm[L.size + cl] = L.We[c];
                    pm[2 * L.size + cl] = L.Wn[c];
                }
            }
            __syncthreads();
            S = &s_sub;
        }
        const long long o0 = B.loff[0];
        const T *m0 = w.lm + o0, *We0 = w.lWe + o0, *Wn0 = w.lWn + o0;
        T* r = w.lb + o0;
        T* z = w.lx + o0;
        T* xi = w.xi + off;
        T* p = w.p + off;
        T* q = w.q + off;
        double rz_old = 0.0, beta = 0.0, pscale = 1.0, rr = 0.0, rr_ref = 1.0, gamma = 0.0, corr = 0.0;
        double rho_last = 1.0, best = 1e300;
        int done = 0, stall = 0, restart = 0;

        // true FP64 residual, stop rule, re-scaled inner residual
        auto check = [&](bool force) {
            if (!force) {
                cells<NT, 8>(
                    n, [&](int c) { return V2<double>{E[c], (double)xi[c]}; },
                    [&](int c, const V2<double>& v) {
                        E[c] = v.a + corr * v.b;
                        xi[c] = T(0);
                    });
                __syncthreads();
            }
            double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            struct Res {
                double e, ee, ew, en, es, we, ww, wn, ws, bb, mm, dV, sv;
                int i, j;
            };
            cells<NT, 2>(
                n,
                [&](int c) {
                    Res v;
                    v.i = c % nx;
                    v.j = c / nx;
                    v.e = E[c];
                    v.ee = v.i + 1 < nx ? E[c + 1] : 0.0;
                    v.ew = v.i > 0 ? E[c - 1] : 0.0;
                    v.en = v.j + 1 < ny ? E[c + nx] : 0.0;
                    v.es = v.j > 0 ? E[c - nx] : 0.0;
                    v.we = We64[c];
                    v.ww = v.i > 0 ? We64[c - 1] : 0.0;
                    v.wn = Wn64[c];
                    v.ws = v.j > 0 ? Wn64[c - nx] : 0.0;
                    v.bb = rhs[c];
                    v.mm = m64[c];
                    v.dV = g.vx[v.i] * g.vy[v.j];
                    v.sv = s64[c];
                    return v;
                },
                [&](int c, const Res& v) {
                    double flux = 0.0;
                    if (v.i + 1 < nx) flux += v.we * (v.e - v.ee);
                    if (v.i > 0) flux += v.ww * (v.e - v.ew);
                    if (v.j + 1 < ny) flux += v.wn * (v.e - v.en);
                    if (v.j > 0) flux += v.ws * (v.e - v.es);
                    const double res = v.bb - v.mm * v.e - flux;
                    r64[c] = res;
                    a[0] += (res / v.dV) * (res / v.dV);
                    a[1] += (v.sv * res) * (v.sv * res);
                    a[2] += (v.bb / v.dV) * (v.bb / v.dV);
                    a[3] += (v.sv * v.bb) * (v.sv * v.bb);
                    a[4] += res * res;
                });
            wg_sum<NT, 5>(a, red);
            const double rrow = a[2] > 0.0 ? sqrt(a[0] / a[2]) : sqrt(a[0]);
            const double rsc = a[3] > 0.0 ? sqrt(a[1] / a[3]) : sqrt(a[1]);
            const double rel = o.norm == 0 ? rrow : rsc;
            rel_row = rrow;
            rel_sc = rsc;
            rel_sel = rel;
            nchecks += 1;
            const double gnew = sqrt(a[4]);
            if (rel < 0.9 * best) {
                best = rel;
                stall = 0;
            } else {
                stall += 1;
            }
            bool demote = false;
            if (!isfinite(rel)) {
                status = ST_EBREAKDOWN;
                done = 1;
            } else if (rel <= o.eps || gnew == 0.0) {
                done = 1;
            } else if (status != ST_OK || iter >= o.max_iter || (!o.reliable && iter > 0) || stall >= 6) {
                if (status == ST_OK && o.reliable) status = ST_ENOCONV;
                done = 1;
            } else {
                const double predicted = gamma * sqrt(rr);
                if (iter > 0 && !(gnew <= 2.0 * predicted)) restart = 1;
                const double ps = gamma > 0.0 ? gamma / gnew : 1.0;
                pscale = ps;
                rz_old *= ps * ps;
                gamma = gnew;
                corr = gnew / mu;
                rho_last = rel;
                rr_ref = 1.0;
                demote = true;
            }
            if (demote) {
                const double ig = 1.0 / gamma;
                cells<NT, 8>(
                    n, [&](int c) { return r64[c]; },
                    [&](int c, double v) {
                        r[c] = (T)(v * ig);
                        xi[c] = T(0);
                    });
                __syncthreads();
            }
        };
        // z = V(r), then r.z and beta
        auto precondition = [&]() {
            b_vcycle<T, NT>(B, w, ainv, S, pool, tile);
            double a[1] = {0.0};
            cells<NT, 8>(
                n, [&](int c) { return V2<T>{r[c], z[c]}; },
                [&](int, const V2<T>& v) { a[0] += (double)v.a * (double)v.b; });
            wg_sum<NT, 1>(a, red);
            const double rz = a[0];
            if (!(rz > 0.0) || !isfinite(rz)) {
                status = ST_EBREAKDOWN;
                done = 1;
            } else {
                beta = iter > 0 ? rz / rz_old : 0.0;
                rz_old = rz;
            }
        };

        check(true);
        if (!done) precondition();
        while (!done) {
            const bool first = iter == 0 || restart;
            const T bt = first ? T(0) : (T)(beta * pscale);
            cells<NT, 8>(
                n, [&](int c) { return V2<T>{z[c], first ? T(0) : p[c]}; },
                [&](int c, const V2<T>& v) { p[c] = first ? v.a : v.a + bt * v.b; });
            __syncthreads();
            double a[1] = {0.0};
            struct Sp {
                T pv, pe, pw, pn, ps, we, ww, wn, ws, mm;
                int i, j;
            };
            cells<NT, 4>(
                n,
                [&](int c) {
                    Sp v;
                    v.i = c % nx;
                    v.j = c / nx;
                    v.pv = p[c];
                    v.pe = v.i + 1 < nx ? p[c + 1] : T(0);
                    v.pw = v.i > 0 ? p[c - 1] : T(0);
                    v.pn = v.j + 1 < ny ? p[c + nx] : T(0);
                    v.ps = v.j > 0 ? p[c - nx] : T(0);
                    v.we = We0[c];
                    v.ww = v.i > 0 ? We0[c - 1] : T(0);
                    v.wn = Wn0[c];
                    v.ws = v.j > 0 ? Wn0[c - nx] : T(0);
                    v.mm = m0[c];
                    return v;
                },
                [&](int c, const Sp& v) {
                    T fl = T(0);
                    if (v.i + 1 < nx) fl += v.we * (v.pv - v.pe);
                    if (v.i > 0) fl += v.ww * (v.pv - v.pw);
                    if (v.j + 1 < ny) fl += v.wn * (v.pv - v.pn);
                    if (v.j > 0) fl += v.ws * (v.pv - v.ps);
                    const T qv = v.mm * v.pv + fl;
                    q[c] = qv;
                    a[0] += (double)v.pv * (double)qv;
                });
            wg_sum<NT, 1>(a, red);
            const double pq = a[0];
            if (!(pq > 0.0) || !isfinite(pq)) {
                status = ST_EBREAKDOWN;
                done = 1;
                break;
            }
            const T al = (T)(rz_old / pq);
            pscale = 1.0;
            restart = 0;
            a[0] = 0.0;
            cells<NT, 8>(
                n, [&](int c) { return V4<T>{xi[c], p[c], r[c], q[c]}; },
                [&](int c, const V4<T>& v) {
                    xi[c] = v.a + al * v.b;
                    const T rn = v.c - al * v.d;
                    r[c] = rn;
                    a[0] += (double)rn * (double)rn;
                });
            wg_sum<NT, 1>(a, red);
            rr = a[0];
            iter += 1;
            bool chk;
            if (o.reliable) {
                const double est = rho_last * sqrt(rr / rr_ref);
                chk = rr < o.delta2 * rr_ref || est <= o.eps;
            } else {
                chk = rr <= o.inner_tol2;
            }
            if (!isfinite(rr)) {
                status = ST_EBREAKDOWN;
                chk = true;
            }
            if (iter >= o.max_iter) chk = true;
            if (chk) check(false);
            if (done) break;
            precondition();
        }
        // final correction with the accumulated inner solution
        cells<NT, 8>(
            n, [&](int c) { return V2<double>{E[c], (double)xi[c]}; },
            [&](int c, const V2<double>& v) {
                E[c] = v.a + corr * v.b;
                xi[c] = T(0);
            });
        if (status == ST_OK && !done) status = ST_ENOCONV;
        // ---- gas update (Section 3.2.1: psi_5, psi_6, psi_11)
        if (o.gas && status == ST_OK) {
            __syncthreads();
            for (int c = t; c < n; c += NT) {
                const double Tn = Tg[c], rho = f.rho[off + c];
                const double CV = rho * f.cv[off + c];
                const double bet = f.kP[off + c] * rho * kC * f.dt;
                const double T3 = Tn * Tn * Tn;
                const double X = 4.0 * bet * kARad * T3;
                Tg[c] = (CV * Tn + 3.0 * bet * kARad * T3 * Tn + bet * E[c]) / (CV + X);
            }
        }
    }
    if (t == 0) {
        BInfo& inf = info[B.id];
        inf.status = status;
        inf.outer_iters = nchecks;
        inf.inner_iters = iter;
        inf.mg_levels = B.nlev;
        inf.rel_resid = rel_sel;
        inf.rel_resid_row = rel_row;
        inf.rel_resid_scaled = rel_sc;
        inf.ms = (float)((double)(wall_clock64() - t_start) / o.clock_khz);
    }
}

}  // namespace fld
