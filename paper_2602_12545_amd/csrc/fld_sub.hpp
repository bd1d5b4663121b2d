// The coarse sub-cycle: the multigrid levels of a grid from some level ls
// down to the coarsest, held in LDS and smoothed by one workgroup (the single
// grid's k_subcycle, and the batched blocks' coarse levels).
#pragma once

#include "fld_line.hpp"

namespace fld {

// ---------------------------------------------------------------------------
// coarse sub-cycle: the V-cycle of all levels >= ls in one workgroup, in LDS
// ---------------------------------------------------------------------------

// threads of the sub-cycle workgroup: binary64 line solves need twice the
// registers, so the binary64 workgroup is half as wide
template <typename T>
constexpr int kSubThreads = sizeof(T) == 4 ? 1024 : 512;
constexpr int kSubMaxLevels = 12;
constexpr int kSubLM = 8;  // cells per lane chunk of the LDS line sweeps

template <typename T>
struct SubLevel {
    int nx, ny;
    const T *m, *We, *Wn;  // row-major inner coefficients (global)
    int off;               // offset of this level's arrays in the LDS pool (elements)
    int tr;                // the level's primary layout is the transposed one
    int pitch;             // LDS row pitch nx + 1 (odd: column walks hit distinct banks)
    int size;              // pitch * ny: elements per LDS array of this level
};

template <typename T>
struct SubCycle {
    int nlev;              // levels ls .. ls + nlev - 1 (the last is the coarsest)
    SubLevel<T> lv[kSubMaxLevels];
    const T* Ainv;         // dense inverse of the coarsest level, cell order of its primary layout
    int bc_off;            // LDS pool offset of the coarsest right-hand side in that cell order
    int part_off;          // LDS pool offset of the coarsest solve's partial sums (one per thread)
    int kcyc;              // 1: K-cycle at the first level (two flexible-CG steps around the V-cycle);
                           // 2: two V-cycles in sequence there, x = c1 + V(b - A c1) (linear)
    int k_off;             // LDS pool offset of the K-cycle arrays (first iterate, its image, partials)
};

// LDS pool per level: m, We, Wn, b, x (5 arrays of pitch * ny; the
// coarsest level's coefficients are not loaded); then the coarsest
// right-hand side in the dense inverse's cell order and one partial sum per
// thread; then, for the K-cycle, two arrays of the first level's size and
// the reduction partials.
//
// One zebra half-sweep of a level in LDS: the lines of parity `par` are
// spread over the workgroup's wavefronts (wave_line_sweep, no barrier inside).
template <typename T, bool ZERO = false, int NT = kSubThreads<T>>
__device__ inline void sub_line(const SubLevel<T>& L, T* pool, bool xdir, int par) {
    const int nx = L.nx, ny = L.ny, P = L.pitch;
    T* m = pool + L.off;
    T* We = m + L.size;
    T* Wn = We + L.size;
    T* b = Wn + L.size;
    T* x = b + L.size;
    const int wave = threadIdx.x >> 6, nw = NT / 64;
    // rows of whole chunks (every power-of-two level from 8 cells) take the
    // path with compile-time chunk bounds: about 40 % fewer instructions for
    // the one or few busy wavefronts that bound a half-sweep
    const int na = xdir ? nx : ny;
    if (wave_line_lanes<kSubLM>(na) * kSubLM == na) {
        if (xdir)
            wave_line_sweep<T, kSubLM, ZERO, true, false, int, true>(nx, ny, par, 1, P, m, We, Wn, b, x, wave, nw);
        else
            wave_line_sweep<T, kSubLM, ZERO, true, false, int, true>(ny, nx, par, P, 1, m, Wn, We, b, x, wave, nw);
    } else if (xdir) {
        wave_line_sweep<T, kSubLM, ZERO, true, false, int>(nx, ny, par, 1, P, m, We, Wn, b, x, wave, nw);
    } else {
        wave_line_sweep<T, kSubLM, ZERO, true, false, int>(ny, nx, par, P, 1, m, Wn, We, b, x, wave, nw);
    }
}

// A x at cell (i, j) of a sub-level in LDS (row pitch P).
template <typename T>
__device__ inline T sub_apply(const T* m, const T* We, const T* Wn, const T* x, int i, int j, int nx, int ny, int P) {
    const int c = j * P + i;
    const T xv = x[c];
    T a = m[c] * xv;
    if (i + 1 < nx) a += We[c] * (xv - x[c + 1]);
    if (i > 0) a += We[c - 1] * (xv - x[c - 1]);
    if (j + 1 < ny) a += Wn[c] * (xv - x[c + P]);
    if (j > 0) a += Wn[c - P] * (xv - x[c - P]);
    return a;
}

// Workgroup sums of NV values (every thread gets them, in one fixed order);
// red holds NV partials per wavefront.
template <typename T, int NV>
__device__ inline void sub_sum(T (&v)[NV], T* red) {
    constexpr int NW = kSubThreads<T> / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NV; ++k)
        for (int o = 32; o >= 1; o >>= 1) v[k] += __shfl_xor(v[k], o);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) red[wave * NV + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        T a = T(0);
        for (int w = 0; w < NW; ++w) a += red[w * NV + k];
        v[k] = a;
    }
    __syncthreads();
}

// The V-cycle over the sub-levels: right-hand side in the first level's b,
// result in its x (every other level's b and x overwritten).
template <typename T, int NT = kSubThreads<T>>
__device__ __forceinline__ void sub_vcycle(const SubCycle<T>& S, T* pool) {
    const int t = threadIdx.x;
    // down
    for (int l = 0; l < S.nlev - 1; ++l) {
        const SubLevel<T>& L = S.lv[l];
        T* x = pool + L.off + 4 * L.size;
        // x starts at zero: the first half-sweep takes zero neighbours, and
        // the first direction's two half-sweeps write every cell
        const bool first_x = !L.tr;  // primary direction first, as on the grid levels
        for (int h = 0; h < 4; ++h) {
            const bool xd = (h < 2) == first_x;
            if (h == 0) sub_line<T, true, NT>(L, pool, xd, 0);
            else sub_line<T, false, NT>(L, pool, xd, h & 1);
            __syncthreads();
        }
        // residual and 2x2 restriction into the next level's b
        const SubLevel<T>& C = S.lv[l + 1];
        const int nc = C.nx * C.ny, P = L.pitch;
        T* m = pool + L.off;
        T* We = m + L.size;
        T* Wn = We + L.size;
        T* b = Wn + L.size;
        T* bc = pool + C.off + 3 * C.size;
        for (int cc = t; cc < nc; cc += NT) {
            const int I = cc % C.nx, J = cc / C.nx;
            T acc = T(0);
            for (int bb = 0; bb < 2; ++bb)
                for (int aa = 0; aa < 2; ++aa) {
                    const int i = 2 * I + aa, j = 2 * J + bb;
                    if (i >= L.nx || j >= L.ny) continue;
                    const int c = j * P + i;
                    const T xv = x[c];
                    T res = b[c] - m[c] * xv;
                    if (i + 1 < L.nx) res -= We[c] * (xv - x[c + 1]);
                    if (i > 0) res -= We[c - 1] * (xv - x[c - 1]);
                    if (j + 1 < L.ny) res -= Wn[c] * (xv - x[c + P]);
                    if (j > 0) res -= Wn[c - P] * (xv - x[c - P]);
                    acc += res;
                }
            bc[J * C.pitch + I] = acc;
        }
        __syncthreads();
    }
    // coarsest: dense inverse in the primary layout's cell order (the
    // right-hand side gathered into that order first).  The inverse is
    // symmetric, so thread r of column group g reads column r: for each c
    // the lanes of a wavefront read consecutive words.  G = NT / n groups
    // split the columns (eight loads in flight per round); their partials
    // are summed in group order.
    {
        const SubLevel<T>& L = S.lv[S.nlev - 1];
        const int n = L.nx * L.ny;
        T* b = pool + L.off + 3 * L.size;
        T* x = b + L.size;
        T* bc = pool + S.bc_off;
        T* part = pool + S.part_off;
        for (int c = t; c < n; c += NT) {
            const int i = L.tr ? c / L.ny : c % L.nx, j = L.tr ? c % L.ny : c / L.nx;
            bc[c] = b[j * L.pitch + i];
        }
        __syncthreads();
        const int G = NT / n, r = t % n, g = t / n;
        if (g < G) {
            const T* col = S.Ainv + r;
            T acc = T(0);
            int c = g;
            for (; c + 7 * G < n; c += 8 * G) {
                T a[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) a[u] = col[(size_t)(c + u * G) * n];
#pragma unroll
                for (int u = 0; u < 8; ++u) acc += a[u] * bc[c + u * G];
            }
            for (; c < n; c += G) acc += col[(size_t)c * n] * bc[c];
            part[t] = acc;
        }
        __syncthreads();
        if (t < n) {
            T acc = part[t];
            for (int q = 1; q < G; ++q) acc += part[q * n + t];
            const int i = L.tr ? t / L.ny : t % L.nx, j = L.tr ? t % L.ny : t / L.nx;
            x[j * L.pitch + i] = acc;
        }
        __syncthreads();
    }
    // up
    for (int l = S.nlev - 2; l >= 0; --l) {
        const SubLevel<T>& L = S.lv[l];
        const SubLevel<T>& C = S.lv[l + 1];
        const int n = L.nx * L.ny;
        T* x = pool + L.off + 4 * L.size;
        const T* xc = pool + C.off + 4 * C.size;
        int i = t % L.nx, j = t / L.nx;
        const int di = NT % L.nx, dj = NT / L.nx;
        for (int c = t; c < n; c += NT) {
            x[j * L.pitch + i] += xc[(j >> 1) * C.pitch + (i >> 1)];
            i += di;
            j += dj;
            if (i >= L.nx) {
                i -= L.nx;
                ++j;
            }
        }
        __syncthreads();
        const bool first_x = !L.tr;
        for (int dir = 0; dir < 2; ++dir) {
            const bool xd = (dir == 0) != first_x;  // reverse order of the pre-smoother
            sub_line<T, false, NT>(L, pool, xd, 1);
            __syncthreads();
            sub_line<T, false, NT>(L, pool, xd, 0);
            __syncthreads();
        }
    }
}

}  // namespace fld
