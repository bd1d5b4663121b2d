// Multigrid-preconditioned CG kernels (inner precision T = float or double).
//
// Inner operator: the assembled E system M divided by mu = max diag(M)
// (one global factor keeps every coefficient and vector inside binary32
// range).  Every level stores its operator as (m, W_e, W_n): the
// non-negative "mass" m (row sum: dV (1 + beta f) plus boundary diagonal
// terms) and the non-negative face conductances to the east / north
// neighbour.  The diagonal m + W_w + W_e + W_s + W_n is a sum of non-negative
// terms, so the rounded operator stays exactly diagonally dominant at every
// level, and matrix-vector products use the flux form m x + sum W (x - x_nb).
//
// Coarse levels: 2x2 aggregation, coarse mass = sum of the four fine masses,
// coarse conductance = omega * (sum of the two fine conductances crossing the
// coarse face); omega = 1 is the Galerkin product P^T M P for piecewise
// constant P, omega = 1/2 rescales it to the coarse spacing.
//
// Smoothers: point red-black Gauss-Seidel, or alternating zebra line
// Gauss-Seidel.  Line solves always run along the rows of a row-major view;
// the other direction uses a transposed copy of the level (coefficients
// transposed once per assembly, vectors transposed between the two sweeps),
// so every load stays coalesced.
#pragma once
#include <type_traits>

#include "fld_kernels.hpp"
#include "fld_line.hpp"
#include "fld_sub.hpp"

namespace fld {

// ---------------------------------------------------------------------------
// hierarchy
// ---------------------------------------------------------------------------

__global__ void k_coarsen(int nx, int ny, const double* __restrict__ m, const double* __restrict__ We,
                          const double* __restrict__ Wn, int nxc, int nyc, double* mc, double* Wec, double* Wnc,
                          double omega) {
    const int I = blockIdx.x * TBX + threadIdx.x;
    const int J = blockIdx.y * TBY + threadIdx.y;
    if (I >= nxc || J >= nyc) return;
    double ms = 0.0, e = 0.0, n = 0.0;
    for (int b = 0; b < 2; ++b) {
        const int j = 2 * J + b;
        if (j >= ny) continue;
        for (int a = 0; a < 2; ++a) {
            const int i = 2 * I + a;
            if (i < nx) ms += m[(size_t)j * nx + i];
        }
        if (2 * I + 2 < nx) e += We[(size_t)j * nx + 2 * I + 1];
    }
    if (2 * J + 2 < ny) {
        for (int a = 0; a < 2; ++a) {
            const int i = 2 * I + a;
            if (i < nx) n += Wn[(size_t)(2 * J + 1) * nx + i];
        }
    }
    const size_t C = (size_t)J * nxc + I;
    mc[C] = ms;
    Wec[C] = omega * e;
    Wnc[C] = omega * n;
}

// Inner-precision copy of a level, divided by mu.
template <typename T>
__global__ void k_demote_level(int n, const double* __restrict__ m, const double* __restrict__ We,
                               const double* __restrict__ Wn, const double* __restrict__ mu, T* mT, T* WeT, T* WnT) {
    const double s = 1.0 / *mu;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        mT[c] = (T)(m[c] * s);
        WeT[c] = (T)(We[c] * s);
        WnT[c] = (T)(Wn[c] * s);
    }
}

// Tiled transpose of up to three [ny][nx] arrays into [nx][ny] arrays,
// 32 x 32 tiles through LDS (padded against bank conflicts).
constexpr int kTT = 32;
template <typename T, int NA>
__global__ __launch_bounds__(256) void k_transpose(int nx, int ny, const T* __restrict__ s0, const T* __restrict__ s1,
                                                   const T* __restrict__ s2, T* __restrict__ d0, T* __restrict__ d1,
                                                   T* __restrict__ d2, const Scalars* __restrict__ sc) {
    if (sc && sc->done) return;
    __shared__ T tile[NA][kTT][kTT + 1];
    const int i0 = blockIdx.x * kTT, j0 = blockIdx.y * kTT;
    const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
    for (int r = ty; r < kTT; r += 8) {
        const int i = i0 + tx, j = j0 + r;
        if (i < nx && j < ny) {
            const size_t c = (size_t)j * nx + i;
            tile[0][r][tx] = s0[c];
            if (NA > 1) tile[NA > 1 ? 1 : 0][r][tx] = s1[c];
            if (NA > 2) tile[NA > 2 ? 2 : 0][r][tx] = s2[c];
        }
    }
    __syncthreads();
    for (int r = ty; r < kTT; r += 8) {
        const int ii = i0 + r, jj = j0 + tx;
        if (ii < nx && jj < ny) {
            const size_t c = (size_t)ii * ny + jj;
            d0[c] = tile[0][tx][r];
            if (NA > 1) d1[c] = tile[NA > 1 ? 1 : 0][tx][r];
            if (NA > 2) d2[c] = tile[NA > 2 ? 2 : 0][tx][r];
        }
    }
}

// Dense inverse of the coarsest level (n <= kCoarseMax cells) in FP64, one
// workgroup.  The cells are numbered along the shorter grid direction first,
// which makes A a band matrix of half-bandwidth w = min(nx, ny) <= BW; its
// Cholesky factor A = L L^T keeps that band (stored by diagonals:
// Lb[i][k] = L(i, i - k), in place of A's band).  One wavefront factors
// column by column (lane r computes L(j + r, j) from the LDS copy of the
// band); then thread j solves L L^T x = e_j, column j of A^-1, keeping the
// last BW unknowns of each substitution in registers (slot = row mod BW).  The
// inverse is stored in the cell order of the view the solver uses on that
// level (`tr`: 0 row-major, 1 transposed).  ywork: n * n doubles (the forward
// solutions).  BW: 4, 8 or 16 (the host picks the smallest >= w).
constexpr int kCoarseMax = 256;
constexpr int kCoarseBand = 16;
template <typename T, int BW>
__global__ __launch_bounds__(kCoarseMax) void k_coarse_setup(int nx, int ny, int tr, const double* __restrict__ m,
                                                             const double* __restrict__ We,
                                                             const double* __restrict__ Wn,
                                                             const double* __restrict__ mu, double* __restrict__ ywork,
                                                             T* __restrict__ Ainv) {
    constexpr int Ld = BW + 1;
    // rows past n (read by the back substitution) stay zero
    __shared__ double Lb[(kCoarseMax + BW) * Ld];
    __shared__ double invd[kCoarseMax];
    const int n = nx * ny, t = threadIdx.x;
    const bool cm = ny < nx;  // band order runs along y first
    const int w = cm ? ny : nx;
    const double s = 1.0 / *mu;
    for (int k = t; k < (kCoarseMax + BW) * Ld; k += kCoarseMax) Lb[k] = 0.0;
    __syncthreads();
    // A's band: A(o, o) and the couplings to the previous cell along the fast
    // direction (o - 1) and to the previous line (o - w; the same cell when w = 1)
    if (t < n) {
        const int o = t;
        const int fi = cm ? o / ny : o % nx, fj = cm ? o % ny : o / nx;  // grid (i, j)
        const int c = fj * nx + fi;
        const double e = (fi + 1 < nx) ? We[c] * s : 0.0, wv = (fi > 0) ? We[c - 1] * s : 0.0;
        const double no = (fj + 1 < ny) ? Wn[c] * s : 0.0, so = (fj > 0) ? Wn[c - nx] * s : 0.0;
        Lb[o * Ld] = m[c] * s + ((wv + e) + (so + no));
        const double fast = cm ? so : wv, line = cm ? wv : so;
        if (w == 1) {
            Lb[o * Ld + 1] = -(fast + line);
        } else {
            Lb[o * Ld + 1] = -fast;
            Lb[o * Ld + w] = -line;
        }
    }
    __syncthreads();
    if (t < 64) {
        for (int j = 0; j < n; ++j) {
            // lane t: A(i, j) - sum_u L(i, j - u) L(j, j - u), i = j + t, u = 1..BW
            // (entries outside the band or before column 0 are zero)
            const int i = min(j + t, n - 1);
            double v = Lb[i * Ld + min(t, BW)], v2 = 0.0;
#pragma unroll
            for (int u = 1; u <= BW; ++u) {
                const double li = (t + u <= BW) ? Lb[i * Ld + min(t + u, BW)] : 0.0;
                if (u & 1) v -= li * Lb[j * Ld + u];
                else v2 -= li * Lb[j * Ld + u];
            }
            v += v2;
            // pivot A(j, j) - ... from lane 0 (the wavefront's first lane) and
            // its reciprocal square root: hardware estimate, two Newton steps
            const unsigned long long vb = __builtin_bit_cast(unsigned long long, v);
            const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)vb);
            const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(vb >> 32));
            const double v0 = __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
            double y = __builtin_amdgcn_rsq(v0);
            y = y * (1.5 - 0.5 * v0 * y * y);
            y = y * (1.5 - 0.5 * v0 * y * y);
            if (t <= w && j + t < n) Lb[i * Ld + t] = v * y;  // lane 0: v0 / sqrt(v0)
            if (t == 0) invd[j] = y;
            // the next column reads this one (same wavefront: LDS keeps the order)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    __syncthreads();
    if (t >= n) return;
    const int j = t;
    double win[BW];
#pragma unroll
    for (int q = 0; q < BW; ++q) win[q] = 0.0;
    // forward: L y = e_j
    for (int ib = 0; ib < n; ib += BW) {
#pragma unroll
        for (int r = 0; r < BW; ++r) {
            const int i = ib + r;
            if (i < n) {
                double acc[4] = {(i == j) ? 1.0 : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k = 1; k <= BW; ++k) acc[k & 3] -= Lb[i * Ld + k] * win[(r - k + BW) % BW];
                const double y = ((acc[0] + acc[1]) + (acc[2] + acc[3])) * invd[i];
                win[r] = y;
                ywork[(size_t)i * n + j] = y;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < BW; ++q) win[q] = 0.0;
    // back: L^T x = y
    auto prim = [&](int o) {  // band-order cell -> index in the solver's cell order
        const int fi = cm ? o / ny : o % nx, fj = cm ? o % ny : o / nx;
        return tr ? fi * ny + fj : fj * nx + fi;
    };
    const int pj = prim(j);
    for (int ib = (n - 1) / BW * BW; ib >= 0; ib -= BW) {
#pragma unroll
        for (int rr = 0; rr < BW; ++rr) {
            const int r = BW - 1 - rr;
            const int i = ib + r;
            if (i < n) {
                double acc[4] = {ywork[(size_t)i * n + j], 0.0, 0.0, 0.0};
#pragma unroll
                for (int k = 1; k <= BW; ++k) acc[k & 3] -= Lb[(i + k) * Ld + k] * win[(r + k) % BW];
                const double x = ((acc[0] + acc[1]) + (acc[2] + acc[3])) * invd[i];
                win[r] = x;
                Ainv[(size_t)prim(i) * n + pj] = (T)x;
            }
        }
    }
}

// Coarsest level: x = A^-1 b with the dense inverse, four lanes per row.
// With DOT (a one-level hierarchy) it also stores r.z as the single partial
// part_rz[0] (k_spmv sums the partials).
constexpr int kCoarseSolveThreads = 4 * kCoarseMax;
template <typename T, bool DOT>
__global__ __launch_bounds__(kCoarseSolveThreads) void k_coarse_solve(int n, const T* __restrict__ Ainv,
                                                                      const T* __restrict__ b, T* __restrict__ x,
                                                                      double* part_rz, Scalars* sc) {
    if (sc->done) return;
    __shared__ T sb[kCoarseMax];
    __shared__ double sh[16];
    const int t = threadIdx.x, row = t >> 2, l4 = t & 3;
    if (t < n) sb[t] = b[t];
    __syncthreads();
    T a = T(0);
    if (row < n) {
        const T* ar = Ainv + (size_t)row * n;
        for (int c = l4; c < n; c += 4) a += ar[c] * sb[c];
    }
    a += __shfl_xor(a, 1, 4);
    a += __shfl_xor(a, 2, 4);
    double acc = 0.0;
    if (row < n && l4 == 0) {
        x[row] = a;
        acc = (double)sb[row] * (double)a;
    }
    if (DOT) {
        const double rz = block_sum(acc, sh);
        if (t == 0) part_rz[0] = rz;
    }
}

// ---------------------------------------------------------------------------
// tiles
// ---------------------------------------------------------------------------

template <int H>
struct TileG {
    static constexpr int LX = TBX + 2 * H;
    static constexpr int LY = TRows + 2 * H;
    static constexpr int N = LX * LY;
};

// Loads m, W_e, W_n of a tile plus halo into LDS (zero outside the grid).
template <typename T, int H>
__device__ inline void load_coef_tile(int nx, int ny, int i0, int j0, const T* m, const T* We, const T* Wn, T* sm,
                                      T* swe, T* swn) {
    constexpr int LX = TileG<H>::LX, N = TileG<H>::N;
    for (int k = ltid(); k < N; k += kThreads) {
        const int lx = k % LX, ly = k / LX, i = i0 + lx - H, j = j0 + ly - H;
        const bool in = (unsigned)i < (unsigned)nx && (unsigned)j < (unsigned)ny;
        const size_t c = (size_t)j * nx + i;
        sm[k] = in ? m[c] : T(0);
        swe[k] = in ? We[c] : T(0);
        swn[k] = in ? Wn[c] : T(0);
    }
}

// ---------------------------------------------------------------------------
// point smoother (red-black Gauss-Seidel, row-major levels)
// ---------------------------------------------------------------------------

// Pre-smoothing from a zero guess (red then black half-sweep), residual on the
// tile, restriction by 2x2 sums.  Halo of 2 cells.
template <typename T>
__global__ __launch_bounds__(256) void k_pre_point(int nx, int ny, const T* __restrict__ b, const T* __restrict__ m,
                                                   const T* __restrict__ We, const T* __restrict__ Wn,
                                                   T* __restrict__ xo, T* __restrict__ bc, int nxc, int nyc,
                                                   const Scalars* __restrict__ sc) {
    if (sc->done) return;
    constexpr int H = 2, LX = TileG<H>::LX, LY = TileG<H>::LY, N = TileG<H>::N;
    __shared__ T sb[N], sm[N], swe[N], swn[N], sx[N];
    __shared__ T sr[TRows][TBX];
    int tbx, tby;
    xcd_tile(tbx, tby);
    const int i0 = tbx * TBX, j0 = tby * TRows, t = ltid();
    load_coef_tile<T, H>(nx, ny, i0, j0, m, We, Wn, sm, swe, swn);
    for (int k = t; k < N; k += kThreads) {
        const int lx = k % LX, ly = k / LX, i = i0 + lx - H, j = j0 + ly - H;
        const bool in = (unsigned)i < (unsigned)nx && (unsigned)j < (unsigned)ny;
        sb[k] = in ? b[(size_t)j * nx + i] : T(0);
    }
    __syncthreads();
    // diagonal needs the west / south conductances: region minus its outer ring
    // (red cells on the ring keep x = 0; they are never read by a tile residual)
    for (int k = t; k < N; k += kThreads) {
        const int lx = k % LX, ly = k / LX, i = i0 + lx - H, j = j0 + ly - H;
        T v = T(0);
        if (lx >= 1 && ly >= 1 && ((i + j) & 1) == 0) {
            const T d = sm[k] + ((swe[k - 1] + swe[k]) + (swn[k - LX] + swn[k]));
            if (d > T(0)) v = sb[k] / d;
        }
        sx[k] = v;
    }
    __syncthreads();
    for (int k = t; k < N; k += kThreads) {
        const int lx = k % LX, ly = k / LX, i = i0 + lx - H, j = j0 + ly - H;
        if (lx < 1 || lx >= LX - 1 || ly < 1 || ly >= LY - 1 || ((i + j) & 1) == 0) continue;
        const T d = sm[k] + ((swe[k - 1] + swe[k]) + (swn[k - LX] + swn[k]));
        const T s = sb[k] + (swe[k] * sx[k + 1] + swe[k - 1] * sx[k - 1] + swn[k] * sx[k + LX] + swn[k - LX] * sx[k - LX]);
        sx[k] = d > T(0) ? s / d : T(0);
    }
    __syncthreads();
    for (int r = 0; r < TRows / TBY; ++r) {
        const int ly = threadIdx.y + r * TBY, lx = threadIdx.x;
        const int i = i0 + lx, j = j0 + ly;
        const int k = (ly + H) * LX + lx + H;
        T res = T(0);
        if (i < nx && j < ny) {
            const T xv = sx[k];
            res = sb[k] - (sm[k] * xv + swe[k] * (xv - sx[k + 1]) + swe[k - 1] * (xv - sx[k - 1]) +
                           swn[k] * (xv - sx[k + LX]) + swn[k - LX] * (xv - sx[k - LX]));
            xo[(size_t)j * nx + i] = xv;
        }
        sr[ly][lx] = res;
    }
    __syncthreads();
    {
        const int cx = t % (TBX / 2), cy = t / (TBX / 2);
        const int I = tbx * (TBX / 2) + cx, J = tby * (TRows / 2) + cy;
        if (cy < TRows / 2 && I < nxc && J < nyc)
            bc[(size_t)J * nxc + I] =
                (sr[2 * cy][2 * cx] + sr[2 * cy][2 * cx + 1]) + (sr[2 * cy + 1][2 * cx] + sr[2 * cy + 1][2 * cx + 1]);
    }
}

// Prolongation (piecewise constant, times omega) + post-smoothing (black then
// red).  With DOT, also accumulates r.z and finalises beta (level 0).
template <typename T, bool DOT>
__global__ __launch_bounds__(256) void k_post_point(int nx, int ny, const T* __restrict__ b, const T* __restrict__ m,
                                                    const T* __restrict__ We, const T* __restrict__ Wn,
                                                    const T* __restrict__ xp, const T* __restrict__ ec, int nxc,
                                                    T omega, T* __restrict__ xo, double* part, Scalars* sc) {
    if (sc->done) return;
    constexpr int H = 2, LX = TileG<H>::LX, LY = TileG<H>::LY, N = TileG<H>::N;
    __shared__ T sb[N], sm[N], swe[N], swn[N], sx[N];
    __shared__ double sh[16];
    int tbx, tby;
    xcd_tile(tbx, tby);
    const int i0 = tbx * TBX, j0 = tby * TRows, t = ltid();
    load_coef_tile<T, H>(nx, ny, i0, j0, m, We, Wn, sm, swe, swn);
    for (int k = t; k < N; k += kThreads) {
        const int lx = k % LX, ly = k / LX, i = i0 + lx - H, j = j0 + ly - H;
        const bool in = (unsigned)i < (unsigned)nx && (unsigned)j < (unsigned)ny;
        const size_t c = (size_t)j * nx + i;
        sb[k] = in ? b[c] : T(0);
        sx[k] = in ? xp[c] + omega * ec[(size_t)(j >> 1) * nxc + (i >> 1)] : T(0);
    }
    __syncthreads();
    for (int k = t; k < N; k += kThreads) {
        const int lx = k % LX, ly = k / LX, i = i0 + lx - H, j = j0 + ly - H;
        if (lx < 1 || lx >= LX - 1 || ly < 1 || ly >= LY - 1 || ((i + j) & 1) == 0) continue;
        if ((unsigned)i >= (unsigned)nx || (unsigned)j >= (unsigned)ny) continue;
        const T d = sm[k] + ((swe[k - 1] + swe[k]) + (swn[k - LX] + swn[k]));
        const T s = sb[k] + (swe[k] * sx[k + 1] + swe[k - 1] * sx[k - 1] + swn[k] * sx[k + LX] + swn[k - LX] * sx[k - LX]);
        sx[k] = d > T(0) ? s / d : T(0);
    }
    __syncthreads();
    double acc = 0.0;
    for (int r = 0; r < TRows / TBY; ++r) {
        const int ly = threadIdx.y + r * TBY, lx = threadIdx.x;
        const int i = i0 + lx, j = j0 + ly;
        if (i >= nx || j >= ny) continue;
        const int k = (ly + H) * LX + lx + H;
        T v = sx[k];
        if (((i + j) & 1) == 0) {
            const T d = sm[k] + ((swe[k - 1] + swe[k]) + (swn[k - LX] + swn[k]));
            const T s =
                sb[k] + (swe[k] * sx[k + 1] + swe[k - 1] * sx[k - 1] + swn[k] * sx[k + LX] + swn[k - LX] * sx[k - LX]);
            v = d > T(0) ? s / d : T(0);
        }
        xo[(size_t)j * nx + i] = v;
        if (DOT) acc += (double)sb[k] * (double)v;
    }
    if (DOT) {
        const double tot = block_sum(acc, sh);
        if (t == 0) part[bid2d()] = tot;
    }
}

// ---------------------------------------------------------------------------
// line smoother (zebra line Gauss-Seidel along rows)
// ---------------------------------------------------------------------------

constexpr int kLineMaxL = 8;    // cells per thread chunk

constexpr int kLineWG = 512;    // threads per workgroup; lines of K chunks, 512/K lines per workgroup
enum { LINE_NORMAL = 0, LINE_ZERO = 1, LINE_PROLONG = 2 };

// One zebra half-sweep: for every row j with j % 2 == par solve exactly
//   (m + W_w + W_e + W_s + W_n) x - W_w x_w - W_e x_e = b + W_s x_s + W_n x_n,
// the south / north rows taken from x (LINE_ZERO: zero, LINE_PROLONG:
// x + omega * coarse correction).  Rows of the other parity are only read, so
// the update is in place.
//
// Parallel tridiagonal solve: a row is split into K chunks of L cells, one
// chunk per thread.  Each thread eliminates its chunk's interior (Thomas,
// three right-hand sides) to express every interior unknown through the last
// unknowns X_{k-1}, X_k of the previous and of its own chunk; substituting the
// neighbour chunk's first row gives one tridiagonal equation per chunk in the
// X's, solved by cyclic reduction (seg_tridiag); back-substitution finishes.
// DOT: partial r.z over the solved rows, stored at part[nb_prev + block]
// (level 0; k_spmv sums the partials).
template <typename T, int MODE, int DOT, bool FULL>
__global__ __launch_bounds__(kLineWG) void k_line(int nx, int ny, int K, int L, int par, const T* __restrict__ m,
                                                  const T* __restrict__ We, const T* __restrict__ Wn,
                                                  const T* __restrict__ b, T* __restrict__ x, const T* __restrict__ ec,
                                                  int nxc, T omega, double* part, int nb_prev, Scalars* sc,
                                                  int* ran) {
    if (sc->done) return;
    if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;  // measurement: this launch did work
    __shared__ T sA[kLineWG], sB[kLineWG], sC[kLineWG], sR[kLineWG];
    __shared__ T sy0[kLineWG], su0[kLineWG], sv0[kLineWG];
    __shared__ double sh[16];
    const int t = threadIdx.x;
    const int lpw = kLineWG / K;
    const int k = t % K;
    // (plain workgroup order: the XCD-aware order measured 1.7 % slower on
    // the 4096-cell rows of the spherical stress grid)
    const int row = 2 * (int)(blockIdx.x * lpw + t / K) + par;
    const bool active = row < ny;
    const int s0 = k * L;
    // FULL: every chunk is exactly kLineMaxL cells inside the row, so the
    // chunk bounds are compile-time constants
    const int Lc = FULL ? kLineMaxL : L;
    const size_t rbase = (size_t)(active ? row : 0) * nx;

    auto xnb = [&](int rr, int g) -> T {  // value of a neighbour-row cell
        const size_t c = (size_t)rr * nx + g;
        if (MODE == LINE_PROLONG) return x[c] + omega * ec[(size_t)(rr >> 1) * nxc + (g >> 1)];
        return x[c];
    };
    // all loads of the chunk first (one memory round trip); cells past the row
    // end become identity rows (d = 1, no couplings, r = 0)
    constexpr int LM = kLineMaxL;
    T vm[LM], vwe[LM], vwn[LM], vws[LM], vb[LM], vxn[LM], vxs[LM];
    const T wwest = (active && s0 > 0 && s0 - 1 < nx) ? We[rbase + s0 - 1] : T(0);
    // full, 16-byte aligned chunk: vector loads (4 x 16 B lanes per wave line)
    constexpr int VW = 16 / sizeof(T);
    const bool vec = active && L == LM && s0 + LM <= nx && ((rbase + s0) % VW) == 0 && (nx % VW) == 0;
    if (vec) {
        const size_t c0 = rbase + s0;
        load_vec<T, LM>(m + c0, vm);
        load_vec<T, LM>(We + c0, vwe);
        load_vec<T, LM>(Wn + c0, vwn);
        load_vec<T, LM>(b + c0, vb);
        if (row > 0) load_vec<T, LM>(Wn + c0 - nx, vws);
        else fill<T, LM>(vws, T(0));
        if (MODE != LINE_ZERO && row + 1 < ny) load_vec<T, LM>(x + c0 + nx, vxn);
        else fill<T, LM>(vxn, T(0));
        if (MODE != LINE_ZERO && row > 0) load_vec<T, LM>(x + c0 - nx, vxs);
        else fill<T, LM>(vxs, T(0));
        if (MODE == LINE_PROLONG) {
#pragma unroll
            for (int q = 0; q < LM; ++q) {
                const int g = s0 + q;
                if (row + 1 < ny) vxn[q] += omega * ec[(size_t)((row + 1) >> 1) * nxc + (g >> 1)];
                if (row > 0) vxs[q] += omega * ec[(size_t)((row - 1) >> 1) * nxc + (g >> 1)];
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < LM; ++q) {
            const int g = s0 + q;
            const bool ok = active && (FULL || (q < Lc && g < nx));
            const size_t cc = rbase + g;
            vm[q] = ok ? m[cc] : T(1);
            vwe[q] = ok ? We[cc] : T(0);
            vwn[q] = ok ? Wn[cc] : T(0);
            vws[q] = (ok && row > 0) ? Wn[cc - nx] : T(0);
            vb[q] = ok ? b[cc] : T(0);
            vxn[q] = (MODE != LINE_ZERO && ok && row + 1 < ny) ? xnb(row + 1, g) : T(0);
            vxs[q] = (MODE != LINE_ZERO && ok && row > 0) ? xnb(row - 1, g) : T(0);
        }
    }
    // keep every load above this point: one round trip instead of a chain
    __builtin_amdgcn_sched_barrier(0);
    // coefficients of chunk cell q: a = -W_w, d, c = -W_e, r
    auto coef = [&](int q, T& a, T& d, T& c, T& r) {
        const T ww = (q == 0) ? wwest : vwe[q > 0 ? q - 1 : 0];
        d = vm[q] + ((ww + vwe[q]) + (vws[q] + vwn[q]));
        a = -ww;
        c = -vwe[q];
        r = vb[q] + vwn[q] * vxn[q] + vws[q] * vxs[q];
    };

    // forward elimination of the chunk interior (local 0 .. L-2)
    T cp[LM], gy[LM], gu[LM], gv[LM];
#pragma unroll
    for (int q = 0; q < LM - 1; ++q) {
        if (q < Lc - 1) {
            T a, d, c, r;
            coef(q, a, d, c, r);
            const T den = (q == 0) ? d : d - a * cp[q > 0 ? q - 1 : 0];
            const T inv = line_rcp(den);
            cp[q] = c * inv;
            gy[q] = ((q == 0) ? r : r - a * gy[q > 0 ? q - 1 : 0]) * inv;
            gu[q] = ((q == 0) ? -a : -a * gu[q > 0 ? q - 1 : 0]) * inv;
            const T rv = (q == Lc - 2) ? -c : T(0);
            gv[q] = ((q == 0) ? rv : rv - a * gv[q > 0 ? q - 1 : 0]) * inv;
        }
    }
    // back substitution: y, u, v overwrite gy, gu, gv
#pragma unroll
    for (int q = LM - 3; q >= 0; --q) {
        if (q < Lc - 2) {
            gy[q] -= cp[q] * gy[q + 1];
            gu[q] -= cp[q] * gu[q + 1];
            gv[q] -= cp[q] * gv[q + 1];
        }
    }
    // interface cell of the chunk (local L-1)
    T aE = T(0), dE = T(1), cE = T(0), rE = T(0);
#pragma unroll
    for (int q = 0; q < LM; ++q)
        if (q == Lc - 1) coef(q, aE, dE, cE, rE);
    T yl = T(0), ul = T(0), vl = T(0);
#pragma unroll
    for (int q = 0; q < LM - 1; ++q)
        if (q == Lc - 2) {
            yl = gy[q];
            ul = gu[q];
            vl = gv[q];
        }
    // the next chunk's first row (y + u X_k + v X_{k+1}), then the K
    // chunk-end unknowns of the row
    const bool has_next = k + 1 < K;
    T yn, un, vn;
    if (K <= 64) {
        const int lane = t & 63;
        yn = __shfl(gy[0], lane + 1, 64);
        un = __shfl(gu[0], lane + 1, 64);
        vn = __shfl(gv[0], lane + 1, 64);
    } else {
        sy0[t] = gy[0];
        su0[t] = gu[0];
        sv0[t] = gv[0];
        __syncthreads();
        yn = has_next ? sy0[t + 1] : T(0);
        un = has_next ? su0[t + 1] : T(0);
        vn = has_next ? sv0[t + 1] : T(0);
    }
    if (!has_next) yn = un = vn = T(0);
    T X, Xp;
    // (sy0 is free again once seg_tridiag's first barrier has passed)
    seg_tridiag<T>(t, k, K, aE * ul, dE + aE * vl + cE * un, cE * vn, rE - aE * yl - cE * yn, sA, sB, sC, sR, sy0, X,
                   Xp);
    double acc = 0.0;
    if (active) {
        T out[LM];
#pragma unroll
        for (int q = 0; q < LM; ++q) {
            out[q] = (q == Lc - 1) ? X : gy[q < LM - 1 ? q : 0] + gu[q < LM - 1 ? q : 0] * Xp +
                                            gv[q < LM - 1 ? q : 0] * X;
            if (DOT && (FULL || (q < Lc && s0 + q < nx))) acc += (double)vb[q] * (double)out[q];
        }
        if (vec) {
            store_vec<T, LM>(x + rbase + s0, out);
        } else {
#pragma unroll
            for (int q = 0; q < LM; ++q)
                if (FULL || (q < Lc && s0 + q < nx)) x[rbase + s0 + q] = out[q];
        }
    }
    if (DOT) {
        const double tot = block_sum(acc, sh);
        if (t == 0) part[nb_prev + blockIdx.x] = tot;
    }
}

// Residual r = b - M x (flux form) on 64 x 16 tiles and restriction by 2x2 sums.
template <typename T>
__global__ __launch_bounds__(256) void k_resid_restrict(int nx, int ny, const T* __restrict__ m,
                                                        const T* __restrict__ We, const T* __restrict__ Wn,
                                                        const T* __restrict__ b, const T* __restrict__ x,
                                                        T* __restrict__ bc, int nxc, int nyc,
                                                        const Scalars* __restrict__ sc) {
    if (sc->done) return;
    constexpr int H = 1, LX = TileG<H>::LX, N = TileG<H>::N;
    __shared__ T sx[N], swe[N], swn[N];
    __shared__ T sr[TRows][TBX];
    int tbx, tby;
    xcd_tile(tbx, tby);
    const int i0 = tbx * TBX, j0 = tby * TRows, t = ltid();
    for (int k = t; k < N; k += kThreads) {
        const int lx = k % LX, ly = k / LX, i = i0 + lx - H, j = j0 + ly - H;
        const bool in = (unsigned)i < (unsigned)nx && (unsigned)j < (unsigned)ny;
        const size_t c = (size_t)j * nx + i;
        sx[k] = in ? x[c] : T(0);
        swe[k] = in ? We[c] : T(0);
        swn[k] = in ? Wn[c] : T(0);
    }
    __syncthreads();
    for (int r = 0; r < TRows / TBY; ++r) {
        const int ly = threadIdx.y + r * TBY, lx = threadIdx.x;
        const int i = i0 + lx, j = j0 + ly;
        const int k = (ly + H) * LX + lx + H;
        T res = T(0);
        if (i < nx && j < ny) {
            const size_t c = (size_t)j * nx + i;
            const T xv = sx[k];
            res = b[c] - (m[c] * xv + swe[k] * (xv - sx[k + 1]) + swe[k - 1] * (xv - sx[k - 1]) +
                          swn[k] * (xv - sx[k + LX]) + swn[k - LX] * (xv - sx[k - LX]));
        }
        sr[ly][lx] = res;
    }
    __syncthreads();
    const int cx = t % (TBX / 2), cy = t / (TBX / 2);
    const int I = tbx * (TBX / 2) + cx, J = tby * (TRows / 2) + cy;
    if (cy < TRows / 2 && I < nxc && J < nyc)
        bc[(size_t)J * nxc + I] =
            (sr[2 * cy][2 * cx] + sr[2 * cy][2 * cx + 1]) + (sr[2 * cy + 1][2 * cx] + sr[2 * cy + 1][2 * cx + 1]);
}

// ---------------------------------------------------------------------------
// CG kernels
// ---------------------------------------------------------------------------

// r.z from the partials of the sweep that produced z, beta = r.z / r.z_old
// (Fletcher-Reeves) or, with rzo (the new residual against the previous
// preconditioned residual, r_k+1 . z_k, summed by k_reduce_rz at rzo[0]),
// beta = max(0, (r.z - r_k+1 . z_k) / r.z_old) (Polak-Ribiere, i.e. flexible
// CG: the multigrid cycles with Krylov levels or a W-type sub-cycle are not a
// fixed symmetric operator); p = z + beta * pscale * p_in (p = z on the first
// iteration or after a restart), q = M p in flux form, partial p.q per
// workgroup (summed by k_update).  pscale and the rescaled r.z_old come from a
// reliable update in between (k_reduce_resid).
template <typename T>
__global__ __launch_bounds__(256) void k_spmv(int nx, int ny, const T* __restrict__ z, const T* __restrict__ pin,
                                              T* __restrict__ pout, T* __restrict__ q, const T* __restrict__ m,
                                              const T* __restrict__ We, const T* __restrict__ Wn,
                                              const double* __restrict__ part_rz, int nrz,
                                              const double* __restrict__ rzo, double* part, Scalars* sc) {
    if (sc->done) return;
    constexpr int H = 1, LX = TileG<H>::LX, N = TileG<H>::N;
    constexpr int NU = (N + kThreads - 1) / kThreads;
    __shared__ T sp[N], swe[N], swn[N];
    __shared__ double sh[16];
    __shared__ double s_rz;
    int tbx, tby;
    xcd_tile(tbx, tby);
    const int i0 = tbx * TBX, j0 = tby * TRows, t = ltid();
    // the tile's loads first; their latency overlaps the r.z sum below
    T zv[NU], pinv[NU], wev[NU], wnv[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int k = t + u * kThreads;
        const int lx = k % LX, ly = k / LX, i = i0 + lx - H, j = j0 + ly - H;
        const bool in = k < N && (unsigned)i < (unsigned)nx && (unsigned)j < (unsigned)ny;
        const size_t c = (size_t)j * nx + i;
        zv[u] = in ? z[c] : T(0);
        pinv[u] = in ? pin[c] : T(0);
        wev[u] = in ? We[c] : T(0);
        wnv[u] = in ? Wn[c] : T(0);
    }
    // r.z of the new preconditioned residual from the partials of the sweep
    // that produced z (every workgroup sums them in the same order, so all
    // agree; workgroup 0 records it), beta = r.z / r.z_old
    {
        double v = 0.0;
        for (int b2 = t; b2 < nrz; b2 += kThreads) v += part_rz[b2];
        const double tot = block_sum(v, sh);
        if (t == 0) s_rz = tot;
        __syncthreads();
    }
    const double rz = s_rz;
    if (!(rz > 0.0) || !isfinite(rz)) {
        if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) {
            sc->status = ST_EBREAKDOWN;
            sc->done = 1;
        }
        return;
    }
    const int iter = sc->iter;
    const bool first = iter == 0 || sc->restart;
    // r_k+1 . z_k belongs to the recurrence residual: after a reliable update
    // replaced r by the true residual (demote set), the Fletcher-Reeves beta
    // with the rescaled r.z_old is taken instead
    const bool flex = rzo != nullptr && !sc->demote;
    const double beta64 = iter == 0 ? 0.0 : flex ? fmax(0.0, (rz - rzo[0]) / sc->rz_old) : rz / sc->rz_old;
    if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) {
        sc->rz_cur = rz;
        sc->beta = beta64;
        sc->apply = 0;  // read by no other kernel of this slot before
    }
    const T beta = first ? T(0) : (T)(beta64 * sc->pscale);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int k = t + u * kThreads;
        if (k < N) {
            sp[k] = first ? zv[u] : zv[u] + beta * pinv[u];
            swe[k] = wev[u];
            swn[k] = wnv[u];
        }
    }
    __syncthreads();
    double acc = 0.0;
    for (int r = 0; r < TRows / TBY; ++r) {
        const int ly = threadIdx.y + r * TBY, lx = threadIdx.x;
        const int i = i0 + lx, j = j0 + ly;
        if (i >= nx || j >= ny) continue;
        const int k = (ly + H) * LX + lx + H;
        const size_t c = (size_t)j * nx + i;
        const T pv = sp[k];
        const T v = m[c] * pv + (swe[k] * (pv - sp[k + 1]) + swe[k - 1] * (pv - sp[k - 1]) +
                                 swn[k] * (pv - sp[k + LX]) + swn[k - LX] * (pv - sp[k - LX]));
        pout[c] = pv;
        q[c] = v;
        acc += (double)pv * (double)v;
    }
    const double tot = block_sum(acc, sh);
    if (t == 0) part[bid2d()] = tot;
}

// alpha = r.z / p.q from the SpMV partials (every workgroup sums them in the
// same order, so all agree; workgroup 0 records the state) -- or, with
// npq = 0, alpha as k_reduce_pq left it (grids with many partials, where
// every workgroup re-reading them costs more than a launch) -- then
// x += alpha p, r -= alpha q and a partial r.r per workgroup into part_rr
// (summed by k_resid64); with zold (the preconditioned residual p was built
// from), also a partial of r_new . zold into part_rzo for the flexible beta;
// workgroup 0 counts the iteration.
template <typename T>
__global__ __launch_bounds__(256) void k_update(int n, T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                                                const T* __restrict__ q, const double* __restrict__ part_pq,
                                                int npq, double* part_rr, const T* __restrict__ zold,
                                                double* part_rzo, Scalars* sc) {
    if (sc->done) return;
    __shared__ double sh[16];
    __shared__ double s_pq;
    if (npq > 0) {
        double v = 0.0;
        for (int b = threadIdx.x; b < npq; b += blockDim.x) v += part_pq[b];
        const double pq = block_sum(v, sh);
        if (threadIdx.x == 0) s_pq = pq;
        __syncthreads();
    }
    T a;
    if (npq > 0) {
        const double pq = s_pq;
        const bool bad = !(pq > 0.0) || !isfinite(pq);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (bad) {
                sc->status = ST_EBREAKDOWN;
                sc->done = 1;
                sc->pending = 1;
            } else {
                sc->alpha = sc->rz_cur / pq;
                sc->iter += 1;
            }
            sc->rz_old = sc->rz_cur;
            sc->pscale = 1.0;
            sc->restart = 0;
            sc->demote = 0;
        }
        if (bad) return;
        a = (T)(sc->rz_cur / pq);
    } else {
        a = (T)sc->alpha;
        if (blockIdx.x == 0 && threadIdx.x == 0) sc->iter += 1;
    }
    // U cells per thread and round, loads first (few workgroups: the
    // memory-level parallelism comes from the unrolling; binary64 measured
    // best without it)
    constexpr int U = sizeof(T) == 4 ? 4 : 1;
    double acc = 0.0, acz = 0.0;
    const bool flex = zold != nullptr;
    const int stride = gridDim.x * blockDim.x;
    for (int c0 = blockIdx.x * blockDim.x + threadIdx.x; c0 < n; c0 += U * stride) {
        T xv[U], pv[U], rv[U], qv[U], zv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = c0 + u * stride;
            const bool ok = c < n;
            xv[u] = ok ? x[c] : T(0);
            pv[u] = ok ? p[c] : T(0);
            rv[u] = ok ? r[c] : T(0);
            qv[u] = ok ? q[c] : T(0);
            zv[u] = ok && flex ? zold[c] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c = c0 + u * stride;
            if (c < n) {
                x[c] = xv[u] + a * pv[u];
                const T rn = rv[u] - a * qv[u];
                r[c] = rn;
                acc += (double)rn * (double)rn;
                acz += (double)rn * (double)zv[u];
            }
        }
    }
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) part_rr[blockIdx.x] = tot;
    if (flex) {
        __syncthreads();
        const double tz = block_sum(acz, sh);
        if (threadIdx.x == 0) part_rzo[blockIdx.x] = tz;
    }
}

// ---------------------------------------------------------------------------
// FP64 refinement
// ---------------------------------------------------------------------------

// E += (gamma / mu) x; x = 0.  Skipped when the assembly flagged a
// non-finite input (err), which leaves E as it entered the solve.
template <typename T>
__global__ __launch_bounds__(256) void k_correct(int n, double* __restrict__ E, T* __restrict__ x,
                                                 const Scalars* __restrict__ sc, int force,
                                                 const int* __restrict__ err) {
    if (*err) return;
    if (!force && (sc->done || !sc->pending)) return;
    const double g = sc->corr;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        E[c] += g * (double)x[c];
        x[c] = T(0);
    }
}

// True residual r = rhs - M E' in flux form, rhs - m E' - sum_f W (E' - E'_nb),
// of the corrected solution E' = E + corr x_inner (evaluated on the fly, the
// same arithmetic as the correction itself; k_apply stores it), and
// per-workgroup partial sums of the stop-rule norms (k_reduce_resid).  The
// forced check at the start of a solve evaluates E itself.
template <typename T>
__global__ __launch_bounds__(256) void k_resid64(Metrics g, const double* __restrict__ E, const T* __restrict__ xin,
                                                 const double* __restrict__ We, const double* __restrict__ Wn,
                                                 const double* __restrict__ m, const double* __restrict__ rhs,
                                                 const double* __restrict__ s, double* __restrict__ r64, double* part,
                                                 const double* __restrict__ part_rr, int nrr, Scalars* sc,
                                                 int force) {
    if (!force && sc->done) return;
    const int nx = g.nx, ny = g.ny;
    constexpr int H = 1, LX = TileG<H>::LX, N = TileG<H>::N;
    constexpr int NS = 5;
    __shared__ double sE[N], sWe[N], sWn[N];
    __shared__ double sh[16];
    __shared__ double s_rr;
    int tbx, tby;
    xcd_tile(tbx, tby);
    const int i0 = tbx * TBX, j0 = tby * TRows, t = ltid();
    if (!force) {
        // recurrence residual r.r from k_update's partials (every workgroup
        // sums them in the same order and takes the same decision; workgroup
        // 0 records it): a reliable update is due when r.r fell by delta since
        // the last one, or predicts the target is met, or at the iteration
        // limit
        double v = 0.0;
        for (int b2 = t; b2 < nrr; b2 += kThreads) v += part_rr[b2];
        const double tot = block_sum(v, sh);
        if (t == 0) s_rr = tot;
        __syncthreads();
        const double rr = s_rr;
        bool check;
        if (sc->reliable) {
            const double est = sc->rho_last * sqrt(rr / sc->rr_ref);
            check = rr < sc->delta2 * sc->rr_ref || est <= sc->eps;
        } else {
            check = rr <= sc->inner_tol2;
        }
        const bool bad = !isfinite(rr);
        if (bad || sc->iter >= sc->max_iter || sc->pending) check = true;
        if (blockIdx.x == 0 && blockIdx.y == 0 && t == 0) {
            sc->rr = rr;
            if (bad) sc->status = ST_EBREAKDOWN;
            if (check) sc->pending = 1;
        }
        if (!check) return;
    }
    const double corr = force ? 0.0 : sc->corr;
    for (int k = t; k < N; k += kThreads) {
        const int lx = k % LX, ly = k / LX, i = i0 + lx - H, j = j0 + ly - H;
        const bool in = (unsigned)i < (unsigned)nx && (unsigned)j < (unsigned)ny;
        const size_t c = (size_t)j * nx + i;
        sE[k] = in ? (force ? E[c] : E[c] + corr * (double)xin[c]) : 0.0;
        sWe[k] = in ? We[c] : 0.0;
        sWn[k] = in ? Wn[c] : 0.0;
    }
    __syncthreads();
    double a[NS] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int r = 0; r < TRows / TBY; ++r) {
        const int ly = threadIdx.y + r * TBY, lx = threadIdx.x;
        const int i = i0 + lx, j = j0 + ly;
        if (i >= nx || j >= ny) continue;
        const int k = (ly + H) * LX + lx + H;
        const size_t c = (size_t)j * nx + i;
        const double e = sE[k];
        double flux = sWe[k] * (e - sE[k + 1]);
        flux += sWe[k - 1] * (e - sE[k - 1]);
        flux += sWn[k] * (e - sE[k + LX]);
        flux += sWn[k - LX] * (e - sE[k - LX]);
        const double b = rhs[c];
        const double res = b - m[c] * e - flux;
        r64[c] = res;
        const double dV = g.vx[i] * g.vy[j];
        const double sv = s[c];
        a[0] += (res / dV) * (res / dV);
        a[1] += (sv * res) * (sv * res);
        a[2] += (b / dV) * (b / dV);
        a[3] += (sv * b) * (sv * b);
        a[4] += res * res;
    }
    double tot[NS];
    for (int q = 0; q < NS; ++q) tot[q] = block_sum(a[q], sh);
    if (t == 0)
        for (int q = 0; q < NS; ++q) part[(size_t)bid2d() * NS + q] = tot[q];
}

// After a true-residual check that did not stop the solve: store the
// corrected solution E += corr_apply x, restart x = 0, and demote the new
// residual r_inner = r / gamma to the inner precision.  (A check that stops the
// solve leaves x for the final correction, which applies the same factor.)
template <typename T>
__global__ __launch_bounds__(256) void k_apply(int n, double* __restrict__ E, const double* __restrict__ r64,
                                               T* __restrict__ r, T* __restrict__ x, const Scalars* __restrict__ sc) {
    if (!sc->apply || sc->done) return;
    const double ig = 1.0 / sc->gamma, g = sc->corr_apply;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        E[c] += g * (double)x[c];
        x[c] = T(0);
        r[c] = (T)(r64[c] * ig);
    }
}

// ---------------------------------------------------------------------------
// scalar reductions: one workgroup sums the producers' partials in a fixed
// order (deterministic) and updates the solver state
// ---------------------------------------------------------------------------

constexpr int kRedThreads = 1024;

__device__ inline double reduce_sum(const double* part, int nb, int stride, int k, double* sh) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) v += part[(size_t)b * stride + k];
    return block_sum(v, sh);
}

// r.z summed once when the last sweep left many partials (one workgroup per
// long line): *out feeds k_spmv as a single partial instead of every SpMV
// workgroup summing all of them
__global__ __launch_bounds__(kRedThreads) void k_reduce_rz(const double* part, int nb, const double* part_rzo,
                                                           int nbo, double* out, const Scalars* sc) {
    if (sc->done) return;
    __shared__ double sh[16];
    const double v = reduce_sum(part, nb, 1, 0, sh);
    if (threadIdx.x == 0) out[0] = v;
    if (part_rzo) {
        const double w = reduce_sum(part_rzo, nbo, 1, 0, sh);
        if (threadIdx.x == 0) out[1] = w;
    }
}

// alpha = r.z / p.q (k_update with npq = 0 reads it from the state instead)
__global__ __launch_bounds__(kRedThreads) void k_reduce_pq(const double* part, int nb, Scalars* sc) {
    if (sc->done) return;
    __shared__ double sh[16];
    const double pq = reduce_sum(part, nb, 1, 0, sh);
    if (threadIdx.x == 0) {
        if (!(pq > 0.0) || !isfinite(pq)) {
            sc->status = ST_EBREAKDOWN;
            sc->done = 1;
            sc->pending = 1;
        } else {
            sc->alpha = sc->rz_cur / pq;
        }
        sc->rz_old = sc->rz_cur;
        sc->pscale = 1.0;
        sc->restart = 0;
        sc->demote = 0;
    }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_resid(const double* part, int nb, const double* mu,
                                                              Scalars* sc, int force) {
    if (!force && (sc->done || !sc->pending)) return;
    constexpr int NS = 5;
    __shared__ double sh[16];
    double tot[NS];
    for (int q = 0; q < NS; ++q) tot[q] = reduce_sum(part, nb, NS, q, sh);
    if (threadIdx.x != 0) return;
    sc->pending = 0;
    sc->corr_apply = force ? 0.0 : sc->corr;  // the correction the residual was evaluated with
    sc->apply = 1;
    for (int q = 0; q < 4; ++q) sc->sums[q] = tot[q];
    const double rrow = tot[2] > 0.0 ? sqrt(tot[0] / tot[2]) : sqrt(tot[0]);
    const double rsc = tot[3] > 0.0 ? sqrt(tot[1] / tot[3]) : sqrt(tot[1]);
    const double rel = sc->norm == 0 ? rrow : rsc;
    sc->rel_row = rrow;
    sc->rel_scaled = rsc;
    sc->rel_sel = rel;
    sc->nchecks += 1;
    const double gnew = sqrt(tot[4]);
    // stagnation: the residual no longer falls (the tolerance is below what
    // binary64 resolves for this system)
    if (rel < 0.9 * sc->best) {
        sc->best = rel;
        sc->stall = 0;
    } else {
        sc->stall += 1;
    }
    if (!isfinite(rel)) {
        sc->status = ST_EBREAKDOWN;
        sc->done = 1;
    } else if (rel <= sc->eps || gnew == 0.0) {
        sc->done = 1;
    } else if (sc->status != ST_OK || sc->iter >= sc->max_iter || (!sc->reliable && sc->iter > 0) || sc->stall >= 6) {
        if (sc->status == ST_OK && sc->reliable) sc->status = ST_ENOCONV;
        sc->done = 1;
    } else {
        // restart the search direction when the true residual is well above the
        // one the (drifted) recurrence predicted
        const double predicted = sc->gamma * sqrt(sc->rr);
        if (sc->iter > 0 && !(gnew <= 2.0 * predicted)) sc->restart = 1;
        const double ps = sc->gamma > 0.0 ? sc->gamma / gnew : 1.0;
        sc->pscale = ps;
        sc->rz_old *= ps * ps;
        sc->gamma = gnew;
        sc->corr = gnew / *mu;
        sc->rho_last = rel;
        sc->rr_ref = 1.0;
        sc->demote = 1;
    }
}

// maximum of the assembly partials (inner-precision normalisation mu)
__global__ __launch_bounds__(kRedThreads) void k_reduce_max(const double* part, int nb, double* mu) {
    __shared__ double sh[16];
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kRedThreads) v = fmax(v, part[b]);
    const double mx = block_max(v, sh);
    if (threadIdx.x == 0) *mu = mx;
}

__global__ void k_zero_int(int* p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

// Per-step record of a captured multi-step run: the solve's final state goes
// to info[counter++] (layout of fld_solve_info).
struct StepInfo {
    int32_t status, outer_iters, inner_iters, mg_levels;
    double rel_resid, rel_resid_row, rel_resid_scaled;
    float ms;
};
__global__ void k_record_step(const Scalars* sc, const int* err, int* counter, int cap, void* info_v, int levels) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int k = *counter;
    if (k < cap) {
        StepInfo* info = static_cast<StepInfo*>(info_v) + k;
        int st = sc->status;
        if (st == ST_OK && !sc->done) st = ST_ENOCONV;
        if (*err) st = ST_ENONFINITE;
        info->status = st;
        info->outer_iters = sc->nchecks;
        info->inner_iters = sc->iter;
        info->mg_levels = levels;
        info->rel_resid = sc->rel_sel;
        info->rel_resid_row = sc->rel_row;
        info->rel_resid_scaled = sc->rel_scaled;
        info->ms = 0.f;
    }
    *counter = k + 1;
}

// Empty kernel: calibration of the cost of a timed launch (event pair).
__global__ void k_noop(int* ran) {
    if (ran && threadIdx.x == 0 && blockIdx.x == 0) *ran = 1;
}

__global__ void k_init_scalars(Scalars* sc, double eps, double delta2, double inner_tol2, int max_iter, int norm,
                               int reliable) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    sc->rz_old = sc->rz_cur = 0.0;
    sc->alpha = sc->beta = 0.0;
    sc->pscale = 1.0;
    sc->rr = 0.0;
    sc->rr_ref = 1.0;
    sc->gamma = 0.0;
    sc->corr = 0.0;
    sc->rho_last = 1.0;
    for (int q = 0; q < 4; ++q) sc->sums[q] = 0.0;
    sc->rel_row = sc->rel_scaled = sc->rel_sel = 0.0;
    sc->eps = eps;
    sc->delta2 = delta2;
    sc->inner_tol2 = inner_tol2;
    sc->iter = 0;
    sc->done = 0;
    sc->pending = 1;
    sc->status = ST_OK;
    sc->max_iter = max_iter;
    sc->norm = norm;
    sc->reliable = reliable;
    sc->nchecks = 0;
    sc->best = 1e300;
    sc->stall = 0;
    sc->restart = 0;
    sc->demote = 0;
    sc->apply = 0;
    sc->corr_apply = 0.0;
}

}  // namespace fld

namespace fld {

template <typename T>
__global__ __launch_bounds__(kSubThreads<T>) void k_subcycle(SubCycle<T> S, const T* __restrict__ bin, T* __restrict__ xout,
                                                          const Scalars* __restrict__ sc) {
    if (sc->done) return;
    extern __shared__ unsigned char smem_raw[];
    T* pool = reinterpret_cast<T*>(smem_raw);
    const int t = threadIdx.x;
    // coefficients of every sub-level but the coarsest (solved by its dense
    // inverse), and the right-hand side of the first
    for (int l = 0; l < S.nlev - 1; ++l) {
        const SubLevel<T>& L = S.lv[l];
        const int n = L.nx * L.ny, z = L.size;
        T* m = pool + L.off;
        // (i, j) of cell c advanced incrementally: no division per cell
        constexpr int NT = kSubThreads<T>;
        int i = t % L.nx, j = t / L.nx;
        const int di = NT % L.nx, dj = NT / L.nx;
        for (int c = t; c < n; c += NT) {
            const int cl = j * L.pitch + i;
            m[cl] = L.m[c];
            m[z + cl] = L.We[c];
            m[2 * z + cl] = L.Wn[c];
            // input in the level's primary layout
            if (l == 0) m[3 * z + cl] = bin[L.tr ? i * L.ny + j : c];
            i += di;
            j += dj;
            if (i >= L.nx) {
                i -= L.nx;
                ++j;
            }
        }
    }
    __syncthreads();
    // K-cycle (Notay and Vassilevski, 2008): the result is the A-norm best
    // combination of c1 = V(b) and c2 = V(b - (c1.b / c1.A c1) A c1); one
    // copy of the V-cycle code serves both passes
    const SubLevel<T>& L0 = S.lv[0];
    const int n0 = L0.nx * L0.ny, z0 = L0.size, P0 = L0.pitch;
    T* m0 = pool + L0.off;
    T* b0 = m0 + 3 * z0;
    T* x0 = m0 + 4 * z0;
    T* c1 = pool + S.k_off;
    T* v1 = c1 + z0;
    T* red = v1 + z0;
    constexpr int NT = kSubThreads<T>;
    const int di = NT % L0.nx, dj = NT / L0.nx;
    constexpr int NW = NT / 64;
    T f1 = T(1), f2 = T(0);  // output = f1 * (c1, or x without K) + f2 * x
    // rho1 and s1 wait in LDS (red[3 NW], red[3 NW + 1]) during the second
    // V-cycle, which needs every register
    for (int pass = 0;; ++pass) {
        sub_vcycle(S, pool);
        if (!S.kcyc) break;
        if (pass == 0 && S.kcyc == 2) {
            // c1 = x; b <- b - A c1 (the second V-cycle solves for the rest)
            int i = t % L0.nx, j = t / L0.nx;
            for (int c = t; c < n0; c += NT) {
                const int cl = j * P0 + i;
                const T av = sub_apply(m0, m0 + z0, m0 + 2 * z0, x0, i, j, L0.nx, L0.ny, P0);
                c1[cl] = x0[cl];
                b0[cl] -= av;
                i += di;
                j += dj;
                if (i >= L0.nx) {
                    i -= L0.nx;
                    ++j;
                }
            }
            __syncthreads();
            continue;
        }
        if (S.kcyc == 2) {  // x = c2: output c1 + c2
            f2 = T(1);
            break;
        }
        if (pass == 0) {
            // c1 = x, v1 = A c1; rho1 = c1.v1, s1 = c1.b / rho1
            T d[2] = {T(0), T(0)};
            int i = t % L0.nx, j = t / L0.nx;
            for (int c = t; c < n0; c += NT) {
                const int cl = j * P0 + i;
                const T xv = x0[cl];
                const T av = sub_apply(m0, m0 + z0, m0 + 2 * z0, x0, i, j, L0.nx, L0.ny, P0);
                c1[cl] = xv;
                v1[cl] = av;
                d[0] += xv * av;
                d[1] += xv * b0[cl];
                i += di;
                j += dj;
                if (i >= L0.nx) {
                    i -= L0.nx;
                    ++j;
                }
            }
            sub_sum<T, 2>(d, red);
            const T rho1 = d[0];
            // rho1 <= 0 only for c1 = 0 (zero right-hand side): the result is c1
            if (!(rho1 > T(0))) break;
            const T s1 = d[1] / rho1;
            if (t == 0) {
                red[3 * NW] = rho1;
                red[3 * NW + 1] = s1;
            }
            i = t % L0.nx;
            j = t / L0.nx;
            for (int c = t; c < n0; c += NT) {
                const int cl = j * P0 + i;
                b0[cl] -= s1 * v1[cl];
                i += di;
                j += dj;
                if (i >= L0.nx) {
                    i -= L0.nx;
                    ++j;
                }
            }
            __syncthreads();
            continue;  // x = c2 next
        }
        // gam = c2.v1, beta = c2.A c2, a2 = c2.r
        T e[3] = {T(0), T(0), T(0)};
        int i = t % L0.nx, j = t / L0.nx;
        for (int c = t; c < n0; c += NT) {
            const int cl = j * P0 + i;
            const T xv = x0[cl];
            e[0] += xv * v1[cl];
            e[1] += xv * sub_apply(m0, m0 + z0, m0 + 2 * z0, x0, i, j, L0.nx, L0.ny, P0);
            e[2] += xv * b0[cl];
            i += di;
            j += dj;
            if (i >= L0.nx) {
                i -= L0.nx;
                ++j;
            }
        }
        sub_sum<T, 3>(e, red);
        const T rho1 = red[3 * NW], s1 = red[3 * NW + 1];
        // A-norm squared of the part of c2 A-orthogonal to c1; within the
        // rounding of its two terms c2 adds nothing
        const T rho2 = e[1] - e[0] * e[0] / rho1;
        const T tiny = sizeof(T) == 4 ? T(1e-5) : T(1e-12);
        f1 = s1;
        if (rho2 > tiny * e[1]) {
            f2 = e[2] / rho2;
            f1 = s1 - e[0] * f2 / rho1;
        }
        break;
    }
    // output in the first level's primary layout
    {
        const T* xo = S.kcyc ? c1 : x0;
        for (int c = t; c < n0; c += NT) {
            const int i = c % L0.nx, j = c / L0.nx;
            const int cl = j * P0 + i;
            xout[L0.tr ? i * L0.ny + j : c] = f1 * xo[cl] + f2 * x0[cl];
        }
    }
}

}  // namespace fld

namespace fld {

// ---------------------------------------------------------------------------
// Krylov-accelerated launched levels (K-cycle at grid levels 1, 3, 5, ...;
// Notay and Vassilevski, 2008): the coarse problem A_l e = r_l of such a level
// l is solved by two flexible-CG steps, each preconditioned by the cycle from
// level l down (launched levels, some of them Krylov-accelerated in turn, then
// the LDS sub-cycle).  After the first pass (c1 = x): v1 = A_l c1,
// rho1 = c1.v1, s1 = c1.r / rho1, r <- r - s1 v1; after the second (c2 = x):
// gam = c2.v1, beta = c2.A_l c2, a2 = c2.r,
// rho2 = beta - gam^2 / rho1, x = (s1 - gam a2 / (rho1 rho2)) c1 + (a2 / rho2) c2.
// Vectors are in the level's primary layout; sums are FP64 partials per
// workgroup, reduced in a fixed order by one workgroup.
// ---------------------------------------------------------------------------

constexpr int kKLThreads = 256;
constexpr int kKLMaxWG = 2048;

struct KLScal {
    double rho1, s1, f1, f2;
};

// A x in flux form at cell (i, j) of a row-major level view.
template <typename T>
__device__ inline double kl_apply(int nx, int ny, const T* __restrict__ m, const T* __restrict__ We,
                                  const T* __restrict__ Wn, const T* __restrict__ x, int i, int j) {
    const size_t c = (size_t)j * nx + i;
    const double xc = (double)x[c];
    double acc = (double)m[c] * xc;
    if (i > 0) acc += (double)We[c - 1] * (xc - (double)x[c - 1]);
    if (i + 1 < nx) acc += (double)We[c] * (xc - (double)x[c + 1]);
    if (j > 0) acc += (double)Wn[c - nx] * (xc - (double)x[c - nx]);
    if (j + 1 < ny) acc += (double)Wn[c] * (xc - (double)x[c + nx]);
    return acc;
}

// STAGE 0: c1 = x, v1 = A x; partials x.v1, x.b.
// STAGE 1: partials x.v1, x.(A x), x.b.
template <typename T, int STAGE>
__global__ __launch_bounds__(kKLThreads) void k_kl_dots(int nx, int ny, const T* __restrict__ m,
                                                        const T* __restrict__ We, const T* __restrict__ Wn,
                                                        const T* __restrict__ x, const T* __restrict__ b,
                                                        T* __restrict__ c1, T* __restrict__ v1,
                                                        double* __restrict__ part, const Scalars* sc) {
    if (sc->done) return;
    __shared__ double sh[kKLThreads / 64];
    const int n = nx * ny;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int c = blockIdx.x * kKLThreads + threadIdx.x; c < n; c += gridDim.x * kKLThreads) {
        const int i = c % nx, j = c / nx;
        const double xv = (double)x[c];
        const double av = kl_apply<T>(nx, ny, m, We, Wn, x, i, j);
        if (STAGE == 0) {
            c1[c] = x[c];
            v1[c] = (T)av;
            d0 += xv * av;
            d1 += xv * (double)b[c];
        } else {
            d0 += xv * (double)v1[c];
            d1 += xv * av;
            d2 += xv * (double)b[c];
        }
    }
    const int G = gridDim.x;
    double s = block_sum(d0, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    s = block_sum(d1, sh);
    if (threadIdx.x == 0) part[G + blockIdx.x] = s;
    if (STAGE == 1) {
        s = block_sum(d2, sh);
        if (threadIdx.x == 0) part[2 * G + blockIdx.x] = s;
    }
}

// The Krylov level's coefficients from the summed partials v (stage 0:
// x.v1, x.b; stage 1: x.v1, x.(A x), x.b): stage 0 sets rho1 and s1, stage 1
// (with rho1, s1 of stage 0) f1 and f2.
template <int STAGE>
__device__ inline void kl_coeffs(const double* v, KLScal& k, int single) {
    if (STAGE == 0) {
        // rho1 <= 0 only for c1 = 0 (zero right-hand side): the result is c1
        const double rho1 = v[0];
        k.rho1 = rho1;
        k.s1 = rho1 > 0.0 ? v[1] / rho1 : 0.0;
        return;
    }
    const double rho1 = k.rho1, s1 = k.s1;
    double f1 = s1, f2 = 0.0;
    if (rho1 > 0.0) {
        // A-norm squared of the part of c2 A-orthogonal to c1; within the
        // rounding of its two terms c2 adds nothing
        const double rho2 = v[1] - v[0] * v[0] / rho1;
        const double tiny = single ? 1e-5 : 1e-12;
        if (rho2 > tiny * v[1]) {
            f2 = v[2] / rho2;
            f1 = s1 - v[0] * f2 / rho1;
        }
    }
    k.f1 = f1;
    k.f2 = f2;
}

// Sums of the G partials of each of the stage's dot products, in a fixed
// order (the result is valid in every thread).
template <int STAGE, int NT>
__device__ inline void kl_sum(const double* part, int G, double* v, double* sh) {
    __shared__ double s_v[3];
    for (int q = 0; q < (STAGE == 0 ? 2 : 3); ++q) {
        double a = 0.0;
        for (int b = threadIdx.x; b < G; b += NT) a += part[(size_t)q * G + b];
        const double t = block_sum(a, sh);
        if (threadIdx.x == 0) s_v[q] = t;
    }
    __syncthreads();
    for (int q = 0; q < (STAGE == 0 ? 2 : 3); ++q) v[q] = s_v[q];
}

template <int STAGE>
__global__ __launch_bounds__(kRedThreads) void k_kl_reduce(const double* part, int G, KLScal* ks, const Scalars* sc,
                                                           int single) {
    if (sc->done) return;
    __shared__ double sh[kRedThreads / 64];
    double v[3];
    kl_sum<STAGE, kRedThreads>(part, G, v, sh);
    if (threadIdx.x != 0) return;
    KLScal k = *ks;
    kl_coeffs<STAGE>(v, k, single);
    *ks = k;
}

// Levels with few partials (G <= kKLFoldMax) skip k_kl_reduce: every
// workgroup of the consumer sums them itself (same order, same result) and
// workgroup 0 stores the coefficients for the next stage.
constexpr int kKLFoldMax = 512;

// r1 <- r1 - s1 v1 (FOLD: s1 from the stage-0 partials)
template <typename T, bool FOLD>
__global__ __launch_bounds__(kKLThreads) void k_kl_axpy(int n, T* __restrict__ b, const T* __restrict__ v1,
                                                        const double* __restrict__ part, int G, KLScal* ks,
                                                        const Scalars* sc) {
    if (sc->done) return;
    double s1d;
    if (FOLD) {
        __shared__ double sh[kKLThreads / 64];
        double v[3];
        kl_sum<0, kKLThreads>(part, G, v, sh);
        KLScal k{};
        kl_coeffs<0>(v, k, 0);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ks->rho1 = k.rho1;
            ks->s1 = k.s1;
        }
        s1d = k.s1;
    } else {
        s1d = ks->s1;
    }
    const T s1 = (T)s1d;
    for (int c = blockIdx.x * kKLThreads + threadIdx.x; c < n; c += gridDim.x * kKLThreads) b[c] -= s1 * v1[c];
}

// x <- f1 c1 + f2 x (FOLD: f1, f2 from the stage-1 partials and rho1, s1)
template <typename T, bool FOLD>
__global__ __launch_bounds__(kKLThreads) void k_kl_combine(int n, T* __restrict__ x, const T* __restrict__ c1,
                                                           const double* __restrict__ part, int G, KLScal* ks,
                                                           const Scalars* sc, int single) {
    if (sc->done) return;
    double f1d, f2d;
    if (FOLD) {
        __shared__ double sh[kKLThreads / 64];
        double v[3];
        kl_sum<1, kKLThreads>(part, G, v, sh);
        KLScal k = *ks;
        kl_coeffs<1>(v, k, single);
        f1d = k.f1;
        f2d = k.f2;
    } else {
        f1d = ks->f1;
        f2d = ks->f2;
    }
    const T f1 = (T)f1d, f2 = (T)f2d;
    for (int c = blockIdx.x * kKLThreads + threadIdx.x; c < n; c += gridDim.x * kKLThreads)
        x[c] = f1 * c1[c] + f2 * x[c];
}

}  // namespace fld
