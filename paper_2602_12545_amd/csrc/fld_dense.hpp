// Exact solve of a coarsest multigrid level too large for one workgroup's
// dense solve (kCoarseMax < n <= kDenseMax cells): its inverse is formed on
// the GPU once per assembly and applied by a product spread over many
// workgroups, a few microseconds per application where a one-workgroup
// iterative sub-cycle takes tens.
//
// The level's operator is block tridiagonal when its cells are taken line by
// line along the shorter grid direction: nb lines of w <= 64 cells, the
// diagonal blocks D_k tridiagonal (couplings along a line), the off-diagonal
// blocks -B_k diagonal (couplings between lines k and k + 1, B_k = diag(b_k)).
// With the forward and backward Schur complements
//   S_0 = D_0,            S_k = D_k - B_{k-1} S_{k-1}^-1 B_{k-1},
//   Q_{nb-1} = D_{nb-1},  Q_k = D_k - B_k Q_{k+1}^-1 B_k,
// the inverse G = A^-1 has the diagonal blocks
//   G_kk = (D_k - B_{k-1} S_{k-1}^-1 B_{k-1} - B_k Q_{k+1}^-1 B_k)^-1
// and, below the diagonal, G_lk = Q_l^-1 B_{l-1} G_{l-1,k} (l > k), which
// follows from block row l of A G = I; the upper blocks are their transposes.
// Every S_k and Q_k is symmetric positive definite and diagonally dominant
// (the level's matrix is an M-matrix with a positive mass term), so
// Gauss-Jordan without pivoting inverts them stably.  All of it runs in FP64;
// G is stored in the inner precision, in block order (unknown a = k w + p),
// and the product maps block order to the level's storage order on the way
// in and out.
#pragma once

#include "fld_mg.hpp"

namespace fld {

constexpr int kDenseMax = 4096;   // largest level solved this way (cells)
constexpr int kDenseW = 64;       // line length bound: min(nx, ny) <= 64 when nx ny <= 4096
constexpr int kDenseThreads = 256;
constexpr int kDenseRows = 8;     // rows of G per workgroup of the product (two per wavefront)
constexpr int kDenseCols = 16;    // columns of a block column per workgroup of the off-diagonal chains

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

// The two Schur chains, one workgroup each: block 0 stores S_k^-1 (k = 0 ..
// nb-2) in SX, block 1 stores Q_k^-1 (k = nb-1 .. 1) in SY (w x w each,
// row-major, at k w^2).  The chain's matrix stays in registers from one
// line to the next.  Dynamic LDS: 3 n + 2 (2 W + 1) doubles (the staged
// coefficients of every line, the pivot buffers).
template <int W, int TS>
__global__ __launch_bounds__((W / TS) * (W / TS)) void k_dense_chain(DenseGeom g, const double* __restrict__ dd,
                                                            const double* __restrict__ aa,
                                                            const double* __restrict__ cc, double* __restrict__ SX,
                                                            double* __restrict__ SY) {
    constexpr int NT = (W / TS) * (W / TS);
    extern __shared__ double dsm[];
    const int w = g.w, nb = g.nb, n = w * nb, nn = w * w, t = threadIdx.x;
    double* sd = dsm;
    double* sa = sd + n;
    double* sc = sa + n;
    double* buf = sc + n;
    for (int e = t; e < n; e += NT) {
        sd[e] = dd[e];
        sa[e] = aa[e];
        sc[e] = cc[e];
    }
    __syncthreads();
    const int ti = t / (W / TS), tj = t % (W / TS);
    const bool fwd = blockIdx.x == 0;
    double* out = fwd ? SX : SY;
    double a[TS][TS];
    for (int s = 0; s + 1 < nb; ++s) {
        const int k = fwd ? s : nb - 1 - s;
        // the eliminated neighbour (line k - 1 forward, k + 1 backward), whose
        // inverse the tiles hold, couples to line k through b_{k-1} or b_k
        const int kb = fwd ? k - 1 : k;
        const double* dk = sd + k * w;
        const double* ak = sa + k * w;
#pragma unroll
        for (int r = 0; r < TS; ++r)
#pragma unroll
            for (int c = 0; c < TS; ++c) {
                const int i = TS * ti + r, j = TS * tj + c;
                double v = i == j ? 1.0 : 0.0;
                if (i < w && j < w) {
                    v = dn_dk(dk, ak, i, j);
                    if (s > 0) v -= sc[kb * w + i] * a[r][c] * sc[kb * w + j];
                }
                a[r][c] = v;
            }
        dn_gj<W, TS>(a, ti, tj, w, buf);
#pragma unroll
        for (int r = 0; r < TS; ++r)
#pragma unroll
            for (int c = 0; c < TS; ++c) {
                const int i = TS * ti + r, j = TS * tj + c;
                if (i < w && j < w) out[(size_t)k * nn + i * w + j] = a[r][c];
            }
    }
}

// Diagonal blocks, one workgroup per line k: G_kk in FP64 (SG) and in the
// inner precision (G, block order, n x n).
template <typename T, int W, int TS>
__global__ __launch_bounds__((W / TS) * (W / TS)) void k_dense_diag(DenseGeom g, const double* __restrict__ dd,
                                                           const double* __restrict__ aa,
                                                           const double* __restrict__ cc,
                                                           const double* __restrict__ SX,
                                                           const double* __restrict__ SY, double* __restrict__ SG,
                                                           T* __restrict__ G) {
    __shared__ double buf[2 * (2 * W + 1)];
    const int w = g.w, nb = g.nb, n = w * nb, nn = w * w, t = threadIdx.x, k = blockIdx.x;
    const int ti = t / (W / TS), tj = t % (W / TS);
    const double* dk = dd + k * w;
    const double* ak = aa + k * w;
    double a[TS][TS];
#pragma unroll
    for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) {
            const int i = TS * ti + r, j = TS * tj + c;
            double v = i == j ? 1.0 : 0.0;
            if (i < w && j < w) {
                v = dn_dk(dk, ak, i, j);
                if (k > 0) {
                    const double* b = cc + (k - 1) * w;
                    v -= b[i] * SX[(size_t)(k - 1) * nn + i * w + j] * b[j];
                }
                if (k + 1 < nb) {
                    const double* b = cc + k * w;
                    v -= b[i] * SY[(size_t)(k + 1) * nn + i * w + j] * b[j];
                }
            }
            a[r][c] = v;
        }
    dn_gj<W, TS>(a, ti, tj, w, buf);
#pragma unroll
    for (int r = 0; r < TS; ++r)
#pragma unroll
        for (int c = 0; c < TS; ++c) {
            const int i = TS * ti + r, j = TS * tj + c;
            if (i < w && j < w) {
                SG[(size_t)k * nn + i * w + j] = a[r][c];
                G[(size_t)(k * w + i) * n + k * w + j] = static_cast<T>(a[r][c]);
            }
        }
}

// Blocks below (and, transposed, above) the diagonal: workgroup (k, c) walks
// down block column k for the columns c kDenseCols .. of its diagonal block,
// X <- Q_l^-1 B_{l-1} X for l = k + 1 .. nb - 1, storing each G_lk and G_kl.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_dense_off(DenseGeom g, const double* __restrict__ cc,
                                                  const double* __restrict__ SY, const double* __restrict__ SG,
                                                  T* __restrict__ G) {
    static_assert(NT == 256, "2 x 2 tiles: 32 row pairs x 8 column pairs");
    constexpr int PER = kDenseW * kDenseW / NT;
    constexpr int C = kDenseCols;
    __shared__ double Yb[kDenseW * kDenseW];
    __shared__ double X[kDenseW * C];
    const int w = g.w, nb = g.nb, n = w * nb, nn = w * w, t = threadIdx.x;
    const int k = blockIdx.x, q0 = blockIdx.y * C, qn = min(C, w - q0);
    for (int e = t; e < w * C; e += NT) {
        const int p = e / C, q = e - p * C;
        X[e] = q < qn ? SG[(size_t)k * nn + p * w + q0 + q] : 0.0;
    }
    // Q_l^-1 (raw) and b_{l-1} of line l in registers, loaded two lines
    // ahead (two register sets, alternating) and used only after the next
    // barrier, so the loads' latency hides behind the products of the two
    // lines before; B_{l-1} scales the rows of X inside the product
    __shared__ double sbv[kDenseW];
    double ya[PER], yb[PER], ba = 0.0, bb = 0.0;
    auto load = [&](double (&y)[PER], double& bv, int l) {
        const double* Y = SY + (size_t)l * nn;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + q * NT;
            if (e < nn) y[q] = Y[e];
        }
        bv = t < w ? cc[(l - 1) * w + t] : 0.0;
    };
    const int rt = t >> 3, ct = t & 7;  // rows 2 rt, 2 rt + 1; columns 2 ct, 2 ct + 1
    const int i0 = 2 * rt, j0 = 2 * ct;
    const bool act = i0 < w && j0 < qn;
    auto step = [&](int l, double (&y)[PER], double& bv) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int e = t + q * NT;
            if (e < nn) Yb[e] = y[q];
        }
        if (t < w) sbv[t] = bv;
        __syncthreads();
        if (l + 2 < nb) load(y, bv, l + 2);
        double a00 = 0.0, a01 = 0.0, a10 = 0.0, a11 = 0.0;
        if (act) {
            const bool two = i0 + 1 < w;
            for (int m = 0; m < w; ++m) {
                const double bm = sbv[m];
                const double y0 = Yb[i0 * w + m], y1 = two ? Yb[(i0 + 1) * w + m] : 0.0;
                const double x0 = X[m * C + j0] * bm, x1 = X[m * C + j0 + 1] * bm;
                a00 += y0 * x0;
                a01 += y0 * x1;
                a10 += y1 * x0;
                a11 += y1 * x1;
            }
        }
        __syncthreads();
        if (act) {
            X[i0 * C + j0] = a00;
            X[i0 * C + j0 + 1] = a01;
            if (i0 + 1 < w) {
                X[(i0 + 1) * C + j0] = a10;
                X[(i0 + 1) * C + j0 + 1] = a11;
            }
        }
        __syncthreads();
        // G_lk: rows l w + p, columns k w + q0 + q; G_kl the transpose
        for (int e = t; e < w * qn; e += NT) {
            const int p = e / qn, q = e - p * qn;
            G[(size_t)(l * w + p) * n + k * w + q0 + q] = static_cast<T>(X[p * C + q]);
        }
        for (int e = t; e < w * qn; e += NT) {
            const int q = e / w, p = e - q * w;
            G[(size_t)(k * w + q0 + q) * n + l * w + p] = static_cast<T>(X[p * C + q]);
        }
    };
    if (k + 1 < nb) load(ya, ba, k + 1);
    if (k + 2 < nb) load(yb, bb, k + 2);
    for (int l = k + 1; l < nb; l += 2) {
        step(l, ya, ba);
        if (l + 1 < nb) step(l + 1, yb, bb);
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
