// Batched implicit radiation step for many independent blocks (static mesh
// refinement blocks in their independent form, Section 3.3: every block sees
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

namespace fld {

constexpr int kBMaxLev = 12;       // multigrid levels per block
constexpr int kBCoarse = 64;       // coarsest level: at most this many cells, inverted densely
constexpr int kBLineL = 8;         // cells per thread chunk in the line solves
constexpr int kBMaxSide = 1024;    // block side limit
constexpr int kBRedDoubles = 128;  // reduction scratch (5 sums x 16 waves)

struct BBlock {
    int nx, ny, nlev, id;          // id: index of the block in the caller's order
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
};

struct BOpts {
    double eps, delta2, inner_tol2, omega;
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
    static constexpr size_t uni = ainv + (size_t)kBCoarse * kBCoarse * sizeof(T);
    static constexpr size_t gj = sizeof(double) * ((size_t)kBCoarse * kBCoarse + kBCoarse);
    static constexpr size_t line = 7 * (size_t)NT * sizeof(T);
    static constexpr size_t bytes = uni + (gj > line ? gj : line);
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

enum { BL_NORMAL = 0, BL_ZERO = 1, BL_PROLONG = 2 };

// One zebra half-sweep of line Gauss-Seidel over a level of one block: every
// line of parity `par` along direction `dir` (0: rows, cells along x; 1:
// columns, cells along y) is solved exactly,
//   (m + sum W) x - W_prev x_prev - W_next x_next = b + W_c- x_c- + W_c+ x_c+,
// with the two neighbour lines taken from x (BL_ZERO: zero; BL_PROLONG: x plus
// the piecewise-constant coarse correction ec).  A line is split into K
// chunks of at most kBLineL cells, one per thread: chunk interiors are
// eliminated locally (three right-hand sides), the K interface unknowns of a
// line are solved by parallel cyclic reduction in LDS, and back-substitution
// completes the chunk.  Lines are processed NT / K at a time.
template <typename T, int NT, int MODE>
__device__ void b_line(int nx, int ny, int dir, int par, const T* __restrict__ m, const T* __restrict__ We,
                       const T* __restrict__ Wn, const T* __restrict__ b, T* __restrict__ x,
                       const T* __restrict__ ec, int nxc, T* lds) {
    const int na = dir ? ny : nx, nlines = dir ? nx : ny;
    const long long sa = dir ? nx : 1, sl = dir ? 1 : nx;
    const T* __restrict__ Wa = dir ? Wn : We;  // coupling to the next cell along the line
    const T* __restrict__ Wc = dir ? We : Wn;  // coupling to the next line
    const int nl = (nlines - par + 1) / 2;
    if (nl <= 0) return;
    int K = 1;
    while (K * kBLineL < na) K <<= 1;
    const int L = max(2, (na + K - 1) / K);
    const int lpp = NT / K;
    T *sA = lds, *sB = lds + NT, *sC = lds + 2 * NT, *sR = lds + 3 * NT;
    T *sy0 = lds + 4 * NT, *su0 = lds + 5 * NT, *sv0 = lds + 6 * NT;
    const int t = threadIdx.x, k = t % K, s0 = k * L;
    constexpr int LM = kBLineL;
    for (int q0 = 0; q0 < nl; q0 += lpp) {
        const int ql = q0 + t / K;
        const bool active = ql < nl;
        const int line = 2 * ql + par;
        const long long lb = (long long)(active ? line : 0) * sl;
        auto coarse = [&](int ln, int pos) -> T {
            const int i = dir ? ln : pos, j = dir ? pos : ln;
            return ec[(long long)(j >> 1) * nxc + (i >> 1)];
        };
        T vm[LM], va[LM], vcn[LM], vcs[LM], vb[LM], vxn[LM], vxs[LM];
        const T wprev = (active && s0 > 0 && s0 - 1 < na) ? Wa[lb + (long long)(s0 - 1) * sa] : T(0);
#pragma unroll
        for (int q = 0; q < LM; ++q) {
            const int g = s0 + q;
            const bool ok = active && q < L && g < na;
            const long long c = lb + (long long)g * sa;
            vm[q] = ok ? m[c] : T(1);
            va[q] = ok ? Wa[c] : T(0);
            vcn[q] = ok ? Wc[c] : T(0);
            vcs[q] = (ok && line > 0) ? Wc[c - sl] : T(0);
            vb[q] = ok ? b[c] : T(0);
            T xn = T(0), xs = T(0);
            if (MODE != BL_ZERO && ok) {
                if (line + 1 < nlines) {
                    xn = x[c + sl];
                    if (MODE == BL_PROLONG) xn += coarse(line + 1, g);
                }
                if (line > 0) {
                    xs = x[c - sl];
                    if (MODE == BL_PROLONG) xs += coarse(line - 1, g);
                }
            }
            vxn[q] = xn;
            vxs[q] = xs;
        }
        auto coef = [&](int q, T& a, T& d, T& c, T& r) {
            const T wp = (q == 0) ? wprev : va[q > 0 ? q - 1 : 0];
            d = vm[q] + ((wp + va[q]) + (vcs[q] + vcn[q]));
            a = -wp;
            c = -va[q];
            r = vb[q] + vcn[q] * vxn[q] + vcs[q] * vxs[q];
        };
        // chunk interior (local 0 .. L-2): every unknown as y + u X_prev + v X_own
        T cp[LM], gy[LM], gu[LM], gv[LM];
#pragma unroll
        for (int q = 0; q < LM - 1; ++q) {
            if (q < L - 1) {
                T a, d, c, r;
                coef(q, a, d, c, r);
                const T den = (q == 0) ? d : d - a * cp[q > 0 ? q - 1 : 0];
                const T inv = T(1) / den;
                cp[q] = c * inv;
                gy[q] = ((q == 0) ? r : r - a * gy[q > 0 ? q - 1 : 0]) * inv;
                gu[q] = ((q == 0) ? -a : -a * gu[q > 0 ? q - 1 : 0]) * inv;
                const T rv = (q == L - 2) ? -c : T(0);
                gv[q] = ((q == 0) ? rv : rv - a * gv[q > 0 ? q - 1 : 0]) * inv;
            }
        }
#pragma unroll
        for (int q = LM - 3; q >= 0; --q) {
            if (q < L - 2) {
                gy[q] -= cp[q] * gy[q + 1];
                gu[q] -= cp[q] * gu[q + 1];
                gv[q] -= cp[q] * gv[q + 1];
            }
        }
        // interface row (local L-1) in the interface unknowns X_{k-1}, X_k, X_{k+1}
        T aE = T(0), dE = T(1), cE = T(0), rE = T(0);
#pragma unroll
        for (int q = 0; q < LM; ++q)
            if (q == L - 1) coef(q, aE, dE, cE, rE);
        T yl = T(0), ul = T(0), vl = T(0);
#pragma unroll
        for (int q = 0; q < LM - 1; ++q)
            if (q == L - 2) {
                yl = gy[q];
                ul = gu[q];
                vl = gv[q];
            }
        sy0[t] = gy[0];
        su0[t] = gu[0];
        sv0[t] = gv[0];
        __syncthreads();
        const bool has_next = k + 1 < K;
        const T yn = has_next ? sy0[t + 1] : T(0), un = has_next ? su0[t + 1] : T(0);
        const T vn = has_next ? sv0[t + 1] : T(0);
        sA[t] = aE * ul;
        sB[t] = dE + aE * vl + cE * un;
        sC[t] = cE * vn;
        sR[t] = rE - aE * yl - cE * yn;
        __syncthreads();
        for (int st = 1; st < K; st <<= 1) {
            const T a = sA[t], bb = sB[t], c = sC[t], r = sR[t];
            T na_ = T(0), nb_ = bb, nc_ = T(0), nr_ = r;
            if (k - st >= 0) {
                const T al = -a / sB[t - st];
                na_ = al * sA[t - st];
                nb_ += al * sC[t - st];
                nr_ += al * sR[t - st];
            }
            if (k + st < K) {
                const T ga = -c / sB[t + st];
                nc_ = ga * sC[t + st];
                nb_ += ga * sA[t + st];
                nr_ += ga * sR[t + st];
            }
            __syncthreads();
            sA[t] = na_;
            sB[t] = nb_;
            sC[t] = nc_;
            sR[t] = nr_;
            __syncthreads();
        }
        const T X = sR[t] / sB[t];
        __syncthreads();
        sR[t] = X;
        __syncthreads();
        const T Xp = k > 0 ? sR[t - 1] : T(0);
        if (active) {
#pragma unroll
            for (int q = 0; q < LM; ++q) {
                const int g = s0 + q;
                if (q < L && g < na) {
                    const T v = (q == L - 1) ? X
                                             : gy[q < LM - 1 ? q : 0] + gu[q < LM - 1 ? q : 0] * Xp +
                                                   gv[q < LM - 1 ? q : 0] * X;
                    x[lb + (long long)g * sa] = v;
                }
            }
        }
        __syncthreads();
    }
}

// Residual b - A x (flux form) of a level summed over 2x2 aggregates: the
// right-hand side of the next coarser level.
template <typename T, int NT>
__device__ void b_restrict(int nx, int ny, const T* __restrict__ m, const T* __restrict__ We,
                           const T* __restrict__ Wn, const T* __restrict__ b, const T* __restrict__ x,
                           T* __restrict__ bc, int nxc, int nyc) {
    for (int C = threadIdx.x; C < nxc * nyc; C += NT) {
        const int I = C % nxc, J = C / nxc;
        T sum = T(0);
        for (int j = 2 * J; j < min(2 * J + 2, ny); ++j)
            for (int i = 2 * I; i < min(2 * I + 2, nx); ++i) {
                const long long c = (long long)j * nx + i;
                const T xc = x[c];
                T fl = T(0);
                if (i + 1 < nx) fl += We[c] * (xc - x[c + 1]);
                if (i > 0) fl += We[c - 1] * (xc - x[c - 1]);
                if (j + 1 < ny) fl += Wn[c] * (xc - x[c + nx]);
                if (j > 0) fl += Wn[c - nx] * (xc - x[c - nx]);
                sum += b[c] - m[c] * xc - fl;
            }
        bc[C] = sum;
    }
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
__device__ void b_coarse_solve(int n, const T* ainv, const T* __restrict__ b, T* __restrict__ x) {
    for (int c = threadIdx.x; c < n; c += NT) {
        T s = T(0);
        for (int k = 0; k < n; ++k) s += ainv[c * n + k] * b[k];
        x[c] = s;
    }
    __syncthreads();
}

// z = V(r): one V-cycle from a zero start; r is the fine level's b array and z
// its x array.  Pre-smoothing: rows (even, odd), columns (even, odd); post-
// smoothing in the reverse order, so the preconditioner is symmetric.
template <typename T, int NT>
__device__ void b_vcycle(const BBlock& B, const BWork<T>& w, const T* ainv, T* lds) {
    const int Lv = B.nlev;
    if (Lv == 1) {
        const long long o = B.loff[0];
        b_coarse_solve<T, NT>(B.lnx[0] * B.lny[0], ainv, w.lb + o, w.lx + o);
        return;
    }
    for (int l = 0; l < Lv - 1; ++l) {
        const int nx = B.lnx[l], ny = B.lny[l];
        const long long o = B.loff[l], oc = B.loff[l + 1];
        const T *m = w.lm + o, *We = w.lWe + o, *Wn = w.lWn + o, *b = w.lb + o;
        T* x = w.lx + o;
        b_line<T, NT, BL_ZERO>(nx, ny, 0, 0, m, We, Wn, b, x, nullptr, 0, lds);
        b_line<T, NT, BL_NORMAL>(nx, ny, 0, 1, m, We, Wn, b, x, nullptr, 0, lds);
        b_line<T, NT, BL_NORMAL>(nx, ny, 1, 0, m, We, Wn, b, x, nullptr, 0, lds);
        b_line<T, NT, BL_NORMAL>(nx, ny, 1, 1, m, We, Wn, b, x, nullptr, 0, lds);
        b_restrict<T, NT>(nx, ny, m, We, Wn, b, x, w.lb + oc, B.lnx[l + 1], B.lny[l + 1]);
        __syncthreads();
    }
    {
        const long long o = B.loff[Lv - 1];
        b_coarse_solve<T, NT>(B.lnx[Lv - 1] * B.lny[Lv - 1], ainv, w.lb + o, w.lx + o);
    }
    for (int l = Lv - 2; l >= 0; --l) {
        const int nx = B.lnx[l], ny = B.lny[l];
        const long long o = B.loff[l], oc = B.loff[l + 1];
        const T *m = w.lm + o, *We = w.lWe + o, *Wn = w.lWn + o, *b = w.lb + o;
        T* x = w.lx + o;
        b_line<T, NT, BL_PROLONG>(nx, ny, 1, 1, m, We, Wn, b, x, w.lx + oc, B.lnx[l + 1], lds);
        b_line<T, NT, BL_NORMAL>(nx, ny, 1, 0, m, We, Wn, b, x, nullptr, 0, lds);
        b_line<T, NT, BL_NORMAL>(nx, ny, 0, 1, m, We, Wn, b, x, nullptr, 0, lds);
        b_line<T, NT, BL_NORMAL>(nx, ny, 0, 0, m, We, Wn, b, x, nullptr, 0, lds);
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
    T* lds = reinterpret_cast<T*>(b_smem + Lay::uni);
    double* gjA = reinterpret_cast<double*>(b_smem + Lay::uni);
    double* gjc = gjA + kBCoarse * kBCoarse;

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
                for (int c = t; c < n; c += NT) {
                    E[c] += corr * (double)xi[c];
                    xi[c] = T(0);
                }
                __syncthreads();
            }
            double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            for (int c = t; c < n; c += NT) {
                const int i = c % nx, j = c / nx;
                const double e = E[c];
                double flux = 0.0;
                if (i + 1 < nx) flux += We64[c] * (e - E[c + 1]);
                if (i > 0) flux += We64[c - 1] * (e - E[c - 1]);
                if (j + 1 < ny) flux += Wn64[c] * (e - E[c + nx]);
                if (j > 0) flux += Wn64[c - nx] * (e - E[c - nx]);
                const double bb = rhs[c];
                const double res = bb - m64[c] * e - flux;
                r64[c] = res;
                const double dV = g.vx[i] * g.vy[j];
                const double sv = s64[c];
                a[0] += (res / dV) * (res / dV);
                a[1] += (sv * res) * (sv * res);
                a[2] += (bb / dV) * (bb / dV);
                a[3] += (sv * bb) * (sv * bb);
                a[4] += res * res;
            }
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
                for (int c = t; c < n; c += NT) {
                    r[c] = (T)(r64[c] * ig);
                    xi[c] = T(0);
                }
                __syncthreads();
            }
        };
        // z = V(r), then r.z and beta
        auto precondition = [&]() {
            b_vcycle<T, NT>(B, w, ainv, lds);
            double a[1] = {0.0};
            for (int c = t; c < n; c += NT) a[0] += (double)r[c] * (double)z[c];
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
            for (int c = t; c < n; c += NT) p[c] = first ? z[c] : z[c] + bt * p[c];
            __syncthreads();
            double a[1] = {0.0};
            for (int c = t; c < n; c += NT) {
                const int i = c % nx, j = c / nx;
                const T pv = p[c];
                T fl = T(0);
                if (i + 1 < nx) fl += We0[c] * (pv - p[c + 1]);
                if (i > 0) fl += We0[c - 1] * (pv - p[c - 1]);
                if (j + 1 < ny) fl += Wn0[c] * (pv - p[c + nx]);
                if (j > 0) fl += Wn0[c - nx] * (pv - p[c - nx]);
                const T v = m0[c] * pv + fl;
                q[c] = v;
                a[0] += (double)pv * (double)v;
            }
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
            for (int c = t; c < n; c += NT) {
                xi[c] += al * p[c];
                const T rn = r[c] - al * q[c];
                r[c] = rn;
                a[0] += (double)rn * (double)rn;
            }
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
        for (int c = t; c < n; c += NT) {
            E[c] += corr * (double)xi[c];
            xi[c] = T(0);
        }
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
        inf.ms = 0.f;
    }
}

}  // namespace fld
