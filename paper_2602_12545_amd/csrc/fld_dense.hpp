// Exact solve of a coarsest multigrid level too large for one workgroup's
// dense solve (kCoarseMax < n <= kDenseMax cells): its inverse is formed on
// the GPU once per assembly and applied by a product spread over many
// workgroups, a few microseconds per application where a one-workgroup
// iterative sub-cycle takes tens.
//
// The level's operator is block tridiagonal when its cells are taken line by
// line along the shorter grid direction: nb lines of w <= 64 cells, diagonal
// blocks A_t (tridiagonal: couplings along a line) and off-diagonal blocks
// -C_t between lines t and t + 1 (diagonal: couplings across lines).  The
// inverse G = A^-1 comes from block cyclic reduction, whose sequential depth
// is log2(nb) block inversions where a line-by-line Schur chain takes nb.
// Eliminating the odd lines t of a level (E_t = A_t^-1 C_{t-1}^T,
// F_t = A_t^-1 C_t) leaves the even lines with
//   A'_u = A_2u - C_{2u-1}^T F_{2u-1} - C_2u E_{2u+1},  C'_u = C_2u F_{2u+1},
// again block tridiagonal; its inverse is G restricted to those lines.
// Going back down, block row t of A G = I gives every block of an odd line
// from its two neighbours:
//   G_tj = E_t G_{t-1,j} + F_t G_{t+1,j} (+ A_t^-1 when j = t),
// first for even j (neighbours' blocks known from the level above), then for
// odd j (the even-odd blocks just formed).  Every block inverted is a Schur
// complement of the symmetric positive definite M-matrix A, so Gauss-Jordan
// without pivoting inverts it stably, and the back-substitution only adds
// non-negative terms.  Level 0, whose blocks are tridiagonal and couplings
// diagonal, inverts its lines by Thomas solves and forms the next level by
// scalings, in one kernel.  All of it runs in FP64; G is stored in the inner
// precision, in block order (unknown a = k w + p), and the product maps block
// order to the level's storage order on the way in and out.
#pragma once

#include "fld_mg.hpp"

namespace fld {

constexpr int kDenseMax = 4096;   // largest level solved this way (cells)
constexpr int kDenseW = 64;       // line length bound: min(nx, ny) <= 64 when nx ny <= 4096
constexpr int kDenseThreads = 256;
constexpr int kDenseRows = 8;     // rows of G per workgroup of the product (two per wavefront)

struct DenseGeom {
    int nx, ny;      // the level's grid
    int cols;        // 1: lines are grid columns (ny < nx); 0: grid rows
    int w, nb;       // cells per line and lines (w nb = nx ny)
    int tr;          // storage order of the level's vectors: 0 row-major (j nx + i), 1 transposed (i ny + j)
    const double *m, *We, *Wn;  // FP64 coefficients of the level, row-major
    const double* mu;           // the level's matrix is (m, W) / mu, as in the inner-precision copies
};

// Row-major index of cell p of line k.
__device__ inline int dn_cell(const DenseGeom& g, int k, int p) { return g.cols ? p * g.nx + k : k * g.nx + p; }

// Storage index of the unknown a = k w + p (block order).
__device__ inline int dn_store(const DenseGeom& g, int a) {
    const int k = a / g.w, p = a - k * g.w;
    const int i = g.cols ? k : p, j = g.cols ? p : k;
    return g.tr ? i * g.ny + j : j * g.nx + i;
}

// Per unknown in block order, scaled by 1 / mu: the diagonal of A (mass plus
// every face coupling), the coupling to the next cell of its line (0 at the
// line's end) and to the same cell of the next line (0 on the last line).
__global__ void k_dense_stage(DenseGeom g, double* __restrict__ dd, double* __restrict__ aa, double* __restrict__ cc) {
    const int n = g.w * g.nb;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const int k = a / g.w, p = a - k * g.w;
    const double s = 1.0 / *g.mu;
    auto along = [&](int kk, int pp) {
        const int c = dn_cell(g, kk, pp);
        return g.cols ? g.Wn[c] : g.We[c];
    };
    auto cross = [&](int kk, int pp) {
        const int c = dn_cell(g, kk, pp);
        return g.cols ? g.We[c] : g.Wn[c];
    };
    const double an = p + 1 < g.w ? along(k, p) : 0.0, ap = p > 0 ? along(k, p - 1) : 0.0;
    const double cn = k + 1 < g.nb ? cross(k, p) : 0.0, cp = k > 0 ? cross(k - 1, p) : 0.0;
    dd[a] = g.m[dn_cell(g, k, p)] * s + ((ap + an) + (cp + cn)) * s;
    aa[a] = an * s;
    cc[a] = cn * s;
}

// Matrices of the set-up live in registers as TS x TS tiles: thread l of the
// (W/TS)^2 threads of a workgroup holds rows TS ti .. TS ti + TS - 1 and
// columns TS tj .. (ti = l / (W/TS), tj = l % (W/TS)); entries beyond the
// w x w matrix hold the identity.
template <int W, int TS>
__device__ inline void dn_sync() {
    if constexpr ((W / TS) * (W / TS) <= 64) {
        // one wavefront: its LDS accesses complete in order
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// In-place inverse of the tiled w x w matrix by Gauss-Jordan elimination
// without pivoting.  For each pivot the owners of its row and column publish
// them in LDS (buf: 2 (2 W + 1) doubles, alternate halves for consecutive
// pivots), one sync, then every thread updates its tile; the pivot chain
// takes one LDS round trip per pivot (and no workgroup barrier when the tiles
// fit one wavefront).
template <int W, int TS>
__device__ void dn_gj(double (&a)[TS][TS], int ti, int tj, int w, double* buf) {
    for (int pr = 0; pr * TS < w; ++pr) {
#pragma unroll
        for (int pc = 0; pc < TS; ++pc) {
            const int p = TS * pr + pc;
            if (p >= w) break;
            double* rb = buf + (p & 1) * (2 * W + 1);
            double* cb = rb + W;
            const bool prow = ti == pr, pcol = tj == pr;
            if (prow) {
#pragma unroll
                for (int c = 0; c < TS; ++c) rb[TS * tj + c] = a[pc][c];
            }
            if (pcol) {
#pragma unroll
                for (int r = 0; r < TS; ++r) cb[TS * ti + r] = a[r][pc];
            }
            dn_sync<W, TS>();
            double rv[TS], cv[TS];
#pragma unroll
            for (int q = 0; q < TS; ++q) {
                rv[q] = rb[TS * tj + q];
                cv[q] = cb[TS * ti + q];
            }
            // d = 1 / a_pp: hardware reciprocal estimate, two Newton steps
            const double x = rb[p];
            double d = __builtin_amdgcn_rcp(x);
            d = fma(d, fma(-x, d, 1.0), d);
            d = fma(d, fma(-x, d, 1.0), d);
            // a_ij - a_ip (a_pj d) for every entry (one FMA each), then the
            // pivot row (a_pj d), column (-a_ip d) and entry (d) set by
            // their owners
            double vd[TS];
#pragma unroll
            for (int c = 0; c < TS; ++c) vd[c] = rv[c] * d;
#pragma unroll
            for (int r = 0; r < TS; ++r)
#pragma unroll
                for (int c = 0; c < TS; ++c) a[r][c] = fma(-cv[r], vd[c], a[r][c]);
            if (prow) {
#pragma unroll
                for (int c = 0; c < TS; ++c) a[pc][c] = vd[c];
            }
            if (pcol) {
#pragma unroll
                for (int r = 0; r < TS; ++r) a[r][pc] = -cv[r] * d;
                if (prow) a[pc][pc] = d;
            }
        }
    }
}

// Block D_k of A at (i, j) (i, j < w) from the staged coefficients.
__device__ inline double dn_dk(const double* dk, const double* ak, int i, int j) {
    return i == j ? dk[i] : j == i + 1 ? -ak[i] : i == j + 1 ? -ak[j] : 0.0;
}

// Matrices of the reduction are w x w, row-major (leading dimension w), one
// per line or per eliminated line; each one a kernel reads transposed is also
// stored transposed, so every LDS operand is a straight copy (leading
// dimension W).  Workgroups of the reduction have 256 threads holding TS x TS
// register tiles (TS = W / 16).
template <int W>
constexpr size_t dn_lds_bytes() {
    return sizeof(double) * (2 * (size_t)W * W + 2 * (2 * W + 1));
}

// A w x w matrix (leading dimension ldm) staged through registers: all of a
// thread's loads are issued before any is stored to LDS.  Thread l takes
// column l % W of rows l / W + q (256 / W), q < PER, so that a wavefront
// reads whole rows.
template <int W>
struct DnFrag {
    static constexpr int PER = W * W / 256, STEP = 256 / W;
    double v[PER];
    __device__ static inline int col() { return threadIdx.x % W; }
    __device__ static inline int row(int q) { return threadIdx.x / W + STEP * q; }
    __device__ inline void fetch(const double* __restrict__ M, int ldm, int w) {
        const int k = col();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = row(q);
            if (i < w && k < w) v[q] = M[(size_t)i * ldm + k];
        }
    }
    __device__ inline void put(double* S, int w) const {
        const int k = col();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = row(q);
            if (i < w && k < w) S[i * W + k] = v[q];
        }
    }
};

// acc += X Y over k < w, with Xt[k][i] = X[i][k] and Y[k][j] in LDS (leading
// dimension W; the rows k of both beyond w up to the next multiple of four
// hold zeros).  16-byte LDS reads, four k per chunk, the next chunk's reads
// issued before the current chunk's FMAs.
template <int W, int TS>
struct DnChunk {
    double x[4][TS], y[4][TS];
    __device__ inline void load(const double* Xt, const double* Y, int k, int ti, int tj) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < TS; r += 2) {
                const double2 x2 = *reinterpret_cast<const double2*>(Xt + (k + u) * W + TS * ti + r);
                const double2 y2 = *reinterpret_cast<const double2*>(Y + (k + u) * W + TS * tj + r);
                x[u][r] = x2.x;
                x[u][r + 1] = x2.y;
                y[u][r] = y2.x;
                y[u][r + 1] = y2.y;
            }
    }
    __device__ inline void fma_into(double (&acc)[TS][TS]) const {
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int r = 0; r < TS; ++r)
#pragma unroll
                for (int c = 0; c < TS; ++c) acc[r][c] = fma(x[u][r], y[u][c], acc[r][c]);
    }
};

template <int W, int TS>
__device__ inline void dn_mm(const double* Xt, const double* Y, int w, int ti, int tj, double (&acc)[TS][TS]) {
    static_assert(TS % 2 == 0 && W % 4 == 0, "pairs of doubles, chunks of four");
    const int nk = (w + 3) / 4;
    DnChunk<W, TS> ca, cb;
    ca.load(Xt, Y, 0, ti, tj);
    for (int c = 0; c < nk; c += 2) {
        if (c + 1 < nk) cb.load(Xt, Y, 4 * (c + 1), ti, tj);
        ca.fma_into(acc);
        if (c + 1 < nk) {
            if (c + 2 < nk) ca.load(Xt, Y, 4 * (c + 2), ti, tj);
            cb.fma_into(acc);
        }
    }
}

// Zeros over the two LDS operands, so that the rows and columns beyond w
// read by the chunked products stay zero (every later copy writes only the
// w x w part).
template <int W>
__device__ inline void dn_lds_zero(double* S) {
    for (int e = threadIdx.x; e < 2 * W * W; e += 256) S[e] = 0.0;
}

// Register tiles of a w x w matrix (leading dimension ldm); beyond w the
// identity (unit) or zero.
template <int TS>
__device__ inline void dn_tile_load(double (&a)[TS][TS], const double* __restrict__ M, int ldm, int w, int ti, int tj,
                                    bool unit) {
#pragma unroll
    for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) {
            const int i = TS * ti + r, j = TS * tj + c;
            a[r][c] = i < w && j < w ? M[(size_t)i * ldm + j] : (unit && i == j ? 1.0 : 0.0);
        }
}

template <typename T, int TS>
__device__ inline void dn_tile_store(const double (&a)[TS][TS], T* __restrict__ M, int ldm, int w, int ti, int tj,
                                     bool trans) {
#pragma unroll
    for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) {
            const int i = TS * ti + r, j = TS * tj + c;
            if (i < w && j < w) M[trans ? (size_t)j * ldm + i : (size_t)i * ldm + j] = static_cast<T>(a[r][c]);
        }
}

template <int TS>
__device__ inline void dn_zero(double (&a)[TS][TS]) {
#pragma unroll
    for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) a[r][c] = 0.0;
}

// M (leading dimension ldm) = the tile matrix transposed, staged through the
// LDS array S (W x W, free on entry: the caller syncs before) so that the
// global stores run along rows; S is in use until the caller's next sync.
template <typename T, int W, int TS>
__device__ inline void dn_store_t(const double (&a)[TS][TS], double* S, T* __restrict__ M, int ldm, int w, int ti,
                                  int tj) {
#pragma unroll
    for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) S[(TS * tj + c) * W + TS * ti + r] = a[r][c];
    __syncthreads();
    const int k = DnFrag<W>::col();
#pragma unroll
    for (int q = 0; q < DnFrag<W>::PER; ++q) {
        const int i = DnFrag<W>::row(q);
        if (i < w && k < w) M[(size_t)i * ldm + k] = static_cast<T>(S[i * W + k]);
    }
}

// Level 0 of the reduction, one workgroup of two wavefronts per line t
// (lane j: column j).  There A_t is tridiagonal and C_t diagonal, so A_t^-1
// comes from w Thomas solves (one per lane, the pivots computed once per
// wavefront, the lane's column held in registers) and every product of the
// reduction is a scaling of its entries.  Odd t: A_t^-1 and its transpose
// into slot (t - 1) / 2 of Ainv and Ainvt.  Even t = 2 u: the level-1 blocks
//   A'_u = A_t - diag(c_{t-1}) A_{t-1}^-1 diag(c_{t-1})
//              - diag(c_t) A_{t+1}^-1 diag(c_t),
//   C'_u = diag(c_t) A_{t+1}^-1 diag(c_{t+1}) (and C'_u transposed),
// the two inverses solved by the two wavefronts side by side.
template <int W>
__global__ __launch_bounds__(128) void k_bcr_level0(int w, int nb, const double* __restrict__ dd,
                                                    const double* __restrict__ aa, const double* __restrict__ cc,
                                                    double* __restrict__ Ainv, double* __restrict__ Ainvt,
                                                    double* __restrict__ A1, double* __restrict__ C1,
                                                    double* __restrict__ C1t) {
    __shared__ double rm[2][W], gm[2][W];  // per wavefront: 1 / pivot, and a_{i-1} / pivot_{i-1}
    __shared__ double sd[2][W], sa[2][W];  // per wavefront: the line's diagonal and couplings
    __shared__ double part[W * W];         // the second wavefront's term of A'_u, [i][j]
    const int t = blockIdx.x, q = threadIdx.x >> 6, j = threadIdx.x & 63, nn = w * w;
    const bool lane = j < w;
    // the line this wavefront inverts (-1: none)
    const int k = (t & 1) ? (q == 0 ? t : -1) : (q == 0 ? (t >= 1 ? t - 1 : -1) : (t + 1 < nb ? t + 1 : -1));
    double col[W];  // column j of A_k^-1
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    if (k >= 0) {
        // the line's coefficients into LDS, so that the sequential pivot
        // loop waits on LDS, not on memory
        if (lane) {
            sd[q][j] = dd[(size_t)k * w + j];
            sa[q][j] = aa[(size_t)k * w + j];
        }
        wave_sync();
        const double* d = sd[q];
        const double* a = sa[q];
        if (j == 0) {
            double r = 1.0 / d[0];
            rm[q][0] = r;
            gm[q][0] = 0.0;
            for (int i = 1; i < w; ++i) {
                const double g = a[i - 1] * r;
                r = 1.0 / (d[i] - a[i - 1] * g);
                rm[q][i] = r;
                gm[q][i] = g;
            }
        }
        wave_sync();
        // forward: y_i = [i == j] + g_i y_{i-1}; back: x_i = (y_i + a_i x_{i+1}) / pivot_i
        double y = j == 0 ? 1.0 : 0.0;
        col[0] = y;
#pragma unroll
        for (int i = 1; i < W; ++i)
            if (i < w) {
                y = fma(gm[q][i], y, i == j ? 1.0 : 0.0);
                col[i] = y;
            }
        double x = 0.0;
#pragma unroll
        for (int i = W - 1; i >= 0; --i)
            if (i < w) {
                x = (i == w - 1 ? col[i] : fma(a[i], x, col[i])) * rm[q][i];
                col[i] = x;
            }
    }
    if (t & 1) {
        // A_t^-1 by columns (coalesced along rows of Ainv), and its
        // transpose through LDS (padded rows) so that Ainvt is also written
        // along rows
        const size_t s = (size_t)(t >> 1) * nn;
        if (q == 0 && lane) {
#pragma unroll
            for (int i = 0; i < W; ++i)
                if (i < w) {
                    Ainv[s + i * w + j] = col[i];
                    part[i * W + j] = col[i];
                }
        }
        __syncthreads();
        for (int r = q; r < w; r += 2)
            if (lane) Ainvt[s + r * w + j] = part[j * W + r];
        return;
    }
    const int u = t >> 1;
    const size_t s = (size_t)u * nn;
    if (q == 1) {
        // diag(c_t) A_{t+1}^-1 diag(c_t) into LDS; C'_u and its transpose
        if (k >= 0 && lane) {
            const double* c = cc + (size_t)t * w;
            const bool hc = t + 2 < nb;
            const double cj = c[j], c2j = hc ? cc[(size_t)(t + 1) * w + j] : 0.0;
#pragma unroll
            for (int i = 0; i < W; ++i)
                if (i < w) {
                    part[i * W + j] = c[i] * col[i] * cj;
                    if (hc) C1[s + i * w + j] = c[i] * col[i] * c2j;
                }
        } else if (lane) {
            for (int i = 0; i < w; ++i) part[i * W + j] = 0.0;
        }
    }
    __syncthreads();
    if (q == 0 && lane) {
        const double* c = t >= 1 ? cc + (size_t)(t - 1) * w : nullptr;
        const double cj = c != nullptr ? c[j] : 0.0;
#pragma unroll
        for (int i = 0; i < W; ++i)
            if (i < w) {
                double v = dn_dk(dd + (size_t)t * w, aa + (size_t)t * w, i, j) - part[i * W + j];
                if (c != nullptr) v -= c[i] * col[i] * cj;
                A1[s + i * w + j] = v;
            }
    }
    if (t + 2 < nb) {
        // C'_u transposed: the second wavefront restages C'_u in LDS once the
        // first has read its term, then both write C'_u^T along rows
        __syncthreads();
        if (q == 1 && lane) {
            const double* c = cc + (size_t)t * w;
            const double c2j = cc[(size_t)(t + 1) * w + j];
#pragma unroll
            for (int i = 0; i < W; ++i)
                if (i < w) part[i * W + j] = c[i] * col[i] * c2j;
        }
        __syncthreads();
        for (int r = q; r < w; r += 2)
            if (lane) C1t[s + r * w + j] = part[j * W + r];
    }
}

// Odd lines t = 2 x + 1 of a level of N lines, one workgroup each: A_t^-1,
// E_t and F_t (F_t only when line t + 1 exists), each also stored transposed
// (Et, Ft) for the back-substitution; slot x of the level's arrays.  Ct holds
// the level's C transposed.  Dynamic LDS: dn_lds_bytes<W>().
template <int W, int TS>
__global__ __launch_bounds__(256) void k_bcr_elim(int w, int N, const double* __restrict__ A,
                                                  const double* __restrict__ C, const double* __restrict__ Ct,
                                                  double* __restrict__ Ainv, double* __restrict__ E,
                                                  double* __restrict__ F, double* __restrict__ Et,
                                                  double* __restrict__ Ft) {
    static_assert((W / TS) * (W / TS) == 256, "256 threads, TS x TS tiles");
    extern __shared__ __align__(16) double dsm[];
    double* Xt = dsm;
    double* Y = Xt + W * W;
    double* buf = Y + W * W;
    const int x = blockIdx.x, t = 2 * x + 1, nn = w * w;
    const bool hasF = t + 1 < N;
    dn_lds_zero<W>(dsm);
    const int ti = threadIdx.x / (W / TS), tj = threadIdx.x % (W / TS);
    // the right-hand factors' loads run beside the inversion
    DnFrag<W> y1, y2;
    y1.fetch(Ct + (size_t)(t - 1) * nn, w, w);
    if (hasF) y2.fetch(C + (size_t)t * nn, w, w);
    double a[TS][TS];
    dn_tile_load<TS>(a, A + (size_t)t * nn, w, w, ti, tj, true);
    dn_gj<W, TS>(a, ti, tj, w, buf);
    dn_tile_store<double, TS>(a, Ainv + (size_t)x * nn, w, w, ti, tj, false);
#pragma unroll
    for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) Xt[(TS * tj + c) * W + TS * ti + r] = a[r][c];
    y1.put(Y, w);
    __syncthreads();
    double acc[TS][TS];
    dn_zero<TS>(acc);
    dn_mm<W, TS>(Xt, Y, w, ti, tj, acc);
    dn_tile_store<double, TS>(acc, E + (size_t)x * nn, w, w, ti, tj, false);
    __syncthreads();
    dn_store_t<double, W, TS>(acc, Y, Et + (size_t)x * nn, w, w, ti, tj);
    if (hasF) {
        __syncthreads();
        y2.put(Y, w);
        __syncthreads();
        dn_zero<TS>(acc);
        dn_mm<W, TS>(Xt, Y, w, ti, tj, acc);
        dn_tile_store<double, TS>(acc, F + (size_t)x * nn, w, w, ti, tj, false);
        __syncthreads();
        dn_store_t<double, W, TS>(acc, Y, Ft + (size_t)x * nn, w, w, ti, tj);
    }
}

// Even lines t = 2 u of the level, one workgroup each: A'_u, C'_u and C'_u
// transposed of the next level (E, F: this level's slots).  Dynamic LDS:
// dn_lds_bytes<W>().
template <int W, int TS>
__global__ __launch_bounds__(256) void k_bcr_reduce(int w, int N, const double* __restrict__ A,
                                                    const double* __restrict__ C, const double* __restrict__ Ct,
                                                    const double* __restrict__ E, const double* __restrict__ F,
                                                    double* __restrict__ A2, double* __restrict__ C2,
                                                    double* __restrict__ C2t) {
    static_assert((W / TS) * (W / TS) == 256, "256 threads, TS x TS tiles");
    extern __shared__ __align__(16) double dsm[];
    double* Xt = dsm;
    double* Y = Xt + W * W;
    const int u = blockIdx.x, t = 2 * u, nn = w * w;
    const int ti = threadIdx.x / (W / TS), tj = threadIdx.x % (W / TS);
    const bool lo = t >= 1, hi = t + 1 < N, c2 = t + 2 < N;
    dn_lds_zero<W>(dsm);
    __syncthreads();
    DnFrag<W> fx, fy;
    // C_{t-1}^T F_{t-1} (Xt[k][i] = C_{t-1}[k][i]), then C_t E_{t+1} and
    // C_t F_{t+1} (Xt[k][i] = C_t[i][k] = Ct_t[k][i]); each next operand's
    // loads run beside the current product
    if (lo) {
        fx.fetch(C + (size_t)(t - 1) * nn, w, w);
        fy.fetch(F + (size_t)((t - 2) / 2) * nn, w, w);
    } else if (hi) {
        fx.fetch(Ct + (size_t)t * nn, w, w);
        fy.fetch(E + (size_t)(t / 2) * nn, w, w);
    }
    double acc[TS][TS], p[TS][TS];
    dn_tile_load<TS>(acc, A + (size_t)t * nn, w, w, ti, tj, false);
    dn_zero<TS>(p);
    if (lo) {
        fx.put(Xt, w);
        fy.put(Y, w);
        __syncthreads();
        if (hi) {
            fx.fetch(Ct + (size_t)t * nn, w, w);
            fy.fetch(E + (size_t)(t / 2) * nn, w, w);
        }
        dn_mm<W, TS>(Xt, Y, w, ti, tj, p);
        __syncthreads();
    }
    if (hi) {
        fx.put(Xt, w);
        fy.put(Y, w);
        __syncthreads();
        if (c2) fy.fetch(F + (size_t)(t / 2) * nn, w, w);
        dn_mm<W, TS>(Xt, Y, w, ti, tj, p);
        if (c2) {
            __syncthreads();
            fy.put(Y, w);
            __syncthreads();
            double q[TS][TS];
            dn_zero<TS>(q);
            dn_mm<W, TS>(Xt, Y, w, ti, tj, q);
            dn_tile_store<double, TS>(q, C2 + (size_t)u * nn, w, w, ti, tj, false);
            __syncthreads();
            dn_store_t<double, W, TS>(q, Y, C2t + (size_t)u * nn, w, w, ti, tj);
        }
    }
#pragma unroll
    for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) acc[r][c] -= p[r][c];
    dn_tile_store<double, TS>(acc, A2 + (size_t)u * nn, w, w, ti, tj, false);
}

// The one line left: G_00 = A_0^-1 into Gw (leading dimension n).  Level 0
// always reduces (a dense level has at least two lines), so G's
// inner-precision copy of this block is written by the last
// back-substitution.
template <int W, int TS>
__global__ __launch_bounds__(256) void k_bcr_top(int w, int n, const double* __restrict__ A,
                                                 double* __restrict__ Gw) {
    __shared__ double buf[2 * (2 * W + 1)];
    const int ti = threadIdx.x / (W / TS), tj = threadIdx.x % (W / TS);
    double a[TS][TS];
    dn_tile_load<TS>(a, A, w, w, ti, tj, true);
    dn_gj<W, TS>(a, ti, tj, w, buf);
    dn_tile_store<double, TS>(a, Gw, n, w, ti, tj, false);
}

// Back-substitution over the odd lines t = 2 x + 1 of a level whose lines are
// the original lines t sg, against line j: G_tj = E_t G_{t-1,j} +
// F_t G_{t+1,j}, plus A_t^-1 when j = t.  OE (j = 2 y even): G_tj and
// G_jt = G_tj^T into Gw; G (non-null at the last level when it is a separate
// inner-precision copy) receives the same blocks and the even-even blocks
// read here: G_{t-1,j}, and G_{t+1,j} when t + 1 is the last line.  !OE
// (j = 2 y + 1 >= t): G_tj and its transpose into Gw, or only into G when G
// is non-null.  L0 (level 0, where E_t = A_t^-1 diag(c_{t-1}) and
// F_t = A_t^-1 diag(c_t)): G_tj = A_t^-1 (diag(c_{t-1}) G_{t-1,j} +
// diag(c_t) G_{t+1,j}), one product; Et then holds A_t^-1 transposed and cc
// the level's couplings.  Dynamic LDS: dn_lds_bytes<W>().
template <typename T, int W, int TS, bool OE, bool L0>
__global__ __launch_bounds__(256) void k_bcr_back(int w, int N, int sg, int n, const double* __restrict__ Ainv,
                                                  const double* __restrict__ Et, const double* __restrict__ Ft,
                                                  const double* __restrict__ cc, double* __restrict__ Gw,
                                                  T* __restrict__ G) {
    static_assert((W / TS) * (W / TS) == 256, "256 threads, TS x TS tiles");
    extern __shared__ __align__(16) double dsm[];
    double* Xt = dsm;
    double* Y = Xt + W * W;
    const int x = blockIdx.x, t = 2 * x + 1, j = OE ? 2 * blockIdx.y : 2 * blockIdx.y + 1, nn = w * w;
    if (!OE && t > j) return;
    const int ti = threadIdx.x / (W / TS), tj = threadIdx.x % (W / TS);
    const bool hi = t + 1 < N;
    dn_lds_zero<W>(dsm);
    __syncthreads();
    const size_t col = (size_t)j * sg * w;
    auto blk = [&](int line) { return (size_t)line * sg * w * n + col; };
    DnFrag<W> fx, fy;
    fx.fetch(Et + (size_t)x * nn, w, w);
    fy.fetch(Gw + blk(t - 1), n, w);
    double acc[TS][TS];
    if (!OE && t == j)
        dn_tile_load<TS>(acc, Ainv + (size_t)x * nn, w, w, ti, tj, false);
    else
        dn_zero<TS>(acc);
    if constexpr (L0) {
        // Y = diag(c_{t-1}) G_{t-1,j} + diag(c_t) G_{t+1,j}: one product
        DnFrag<W> fz;
        if (hi) fz.fetch(Gw + blk(t + 1), n, w);
        fx.put(Xt, w);
        const double* c0 = cc + (size_t)(t - 1) * w;
        const double* c1 = cc + (size_t)t * w;
#pragma unroll
        for (int q = 0; q < DnFrag<W>::PER; ++q) {
            const int i = DnFrag<W>::row(q), k = DnFrag<W>::col();
            if (i < w && k < w) Y[i * W + k] = c0[i] * fy.v[q] + (hi ? c1[i] * fz.v[q] : 0.0);
        }
        __syncthreads();
        if (OE && G != nullptr)
#pragma unroll
            for (int q = 0; q < DnFrag<W>::PER; ++q) {
                const int i = DnFrag<W>::row(q), k = DnFrag<W>::col();
                if (i < w && k < w) {
                    G[blk(t - 1) + (size_t)i * n + k] = static_cast<T>(fy.v[q]);
                    if (t + 1 == N - 1) G[blk(t + 1) + (size_t)i * n + k] = static_cast<T>(fz.v[q]);
                }
            }
        dn_mm<W, TS>(Xt, Y, w, ti, tj, acc);
    } else {
        fx.put(Xt, w);
        fy.put(Y, w);
        __syncthreads();
        if (OE && G != nullptr)
#pragma unroll
            for (int q = 0; q < DnFrag<W>::PER; ++q) {
                const int i = DnFrag<W>::row(q), k = DnFrag<W>::col();
                if (i < w && k < w) G[blk(t - 1) + (size_t)i * n + k] = static_cast<T>(fy.v[q]);
            }
        if (hi) {
            fx.fetch(Ft + (size_t)x * nn, w, w);
            fy.fetch(Gw + blk(t + 1), n, w);
        }
        dn_mm<W, TS>(Xt, Y, w, ti, tj, acc);
        if (hi) {
            __syncthreads();
            fx.put(Xt, w);
            fy.put(Y, w);
            __syncthreads();
            if (OE && G != nullptr && t + 1 == N - 1)
#pragma unroll
                for (int q = 0; q < DnFrag<W>::PER; ++q) {
                    const int i = DnFrag<W>::row(q), k = DnFrag<W>::col();
                    if (i < w && k < w) G[blk(t + 1) + (size_t)i * n + k] = static_cast<T>(fy.v[q]);
                }
            dn_mm<W, TS>(Xt, Y, w, ti, tj, acc);
        }
    }
    const size_t tj0 = (size_t)t * sg * w * n + col, jt0 = (size_t)j * sg * w * n + (size_t)t * sg * w;
    const bool mirror = OE || t != j;
    // with a separate inner-precision copy (last level) the odd-odd blocks
    // and the odd-even ones are not read again in FP64: only the even-odd
    // transposes are, by the odd-odd pass
    if (G == nullptr)
        dn_tile_store<double, TS>(acc, Gw + tj0, n, w, ti, tj, false);
    else
        dn_tile_store<T, TS>(acc, G + tj0, n, w, ti, tj, false);
    if (mirror) {
        // the transpose, staged through LDS for row-wise stores
        __syncthreads();
#pragma unroll
        for (int r = 0; r < TS; ++r)
#pragma unroll
            for (int c = 0; c < TS; ++c) Xt[(TS * tj + c) * W + TS * ti + r] = acc[r][c];
        __syncthreads();
        const int k = DnFrag<W>::col();
#pragma unroll
        for (int q = 0; q < DnFrag<W>::PER; ++q) {
            const int i = DnFrag<W>::row(q);
            if (i < w && k < w) {
                const double v = Xt[i * W + k];
                if (G == nullptr || OE) Gw[jt0 + (size_t)i * n + k] = v;
                if (G != nullptr) G[jt0 + (size_t)i * n + k] = static_cast<T>(v);
            }
        }
    }
}

// x = G b on the level: rows of G spread over workgroups (two per
// wavefront, lanes along the row), b gathered into block order in LDS, x
// scattered back to the storage order.  DOT (a one-level hierarchy): also the
// workgroup's partial of r.z = b.x in part_rz[blockIdx.x].
template <typename T, bool DOT>
__global__ __launch_bounds__(kDenseThreads) void k_dense_solve(DenseGeom g, const T* __restrict__ G,
                                                               const T* __restrict__ b, T* __restrict__ x,
                                                               double* __restrict__ part_rz,
                                                               const Scalars* __restrict__ sc) {
    if (sc->done) return;
    __shared__ __align__(16) T sb[kDenseMax];
    __shared__ double sh[16];
    const int n = g.w * g.nb, t = threadIdx.x, lane = t & 63, wv = t >> 6;
    for (int a = t; a < n; a += kDenseThreads) sb[a] = b[dn_store(g, a)];
    __syncthreads();
    double dot = 0.0;
    constexpr int RW = kDenseRows / (kDenseThreads / 64);
#pragma unroll
    for (int r = 0; r < RW; ++r) {
        const int a = blockIdx.x * kDenseRows + wv * RW + r;
        if (a < n) {
            const T* row = G + (size_t)a * n;
            T s0 = T(0), s1 = T(0);
            constexpr int VW = 16 / sizeof(T);
            if (n % (64 * VW) == 0) {
                // 16-byte loads: each lane takes VW consecutive entries per
                // step, four steps in flight
                using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
                const V* rv = reinterpret_cast<const V*>(row);
                const V* bv = reinterpret_cast<const V*>(sb);
                const int nv = n / VW;
#pragma unroll 4
                for (int c = lane; c < nv; c += 64) {
                    const V g = rv[c], x = bv[c];
                    if constexpr (sizeof(T) == 4) {
                        s0 += g.x * x.x + g.y * x.y;
                        s1 += g.z * x.z + g.w * x.w;
                    } else {
                        s0 += g.x * x.x;
                        s1 += g.y * x.y;
                    }
                }
            } else {
                int c = lane;
#pragma unroll 4
                for (; c + 64 < n; c += 128) {
                    s0 += row[c] * sb[c];
                    s1 += row[c + 64] * sb[c + 64];
                }
                if (c < n) s0 += row[c] * sb[c];
            }
            T s = s0 + s1;
            for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
            if (lane == 0) {
                x[dn_store(g, a)] = s;
                dot += (double)sb[a] * (double)s;
            }
        }
    }
    if (DOT) {
        const double rz = block_sum(dot, sh);
        if (t == 0) part_rz[blockIdx.x] = rz;
    }
}

}  // namespace fld
