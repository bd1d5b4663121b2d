// Wavefront-level zebra line solve: the tridiagonal systems of a set of grid
// lines, each owned by K lanes of one wavefront, with no workgroup barrier.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace fld {

// Reciprocal for the inner line solves: the hardware approximation (1 ulp)
// in binary32; in binary64 the approximation refined by two Newton steps
// (full precision).  Keeps the division latency out of the Thomas chains.
template <typename T>
__device__ inline T line_rcp(T d) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_amdgcn_rcpf(d);
    } else {
        T r = __builtin_amdgcn_rcp(d);
        r = r * (T(2) - d * r);
        r = r * (T(2) - d * r);
        return r;
    }
}

// N consecutive values from a 16-byte aligned address with 16-byte loads.
template <typename T, int N>
__device__ inline void load_vec(const T* __restrict__ p, T (&v)[N]) {
    constexpr int VW = 16 / sizeof(T);
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    const V* q = reinterpret_cast<const V*>(p);
#pragma unroll
    for (int k = 0; k < N / VW; ++k) {
        const V w = q[k];
        if constexpr (sizeof(T) == 4) {
            v[4 * k] = w.x; v[4 * k + 1] = w.y; v[4 * k + 2] = w.z; v[4 * k + 3] = w.w;
        } else {
            v[2 * k] = w.x; v[2 * k + 1] = w.y;
        }
    }
}

template <typename T, int N>
__device__ inline void store_vec(T* __restrict__ p, const T (&v)[N]) {
    constexpr int VW = 16 / sizeof(T);
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
    V* q = reinterpret_cast<V*>(p);
#pragma unroll
    for (int k = 0; k < N / VW; ++k) {
        V w;
        if constexpr (sizeof(T) == 4) {
            w.x = v[4 * k]; w.y = v[4 * k + 1]; w.z = v[4 * k + 2]; w.w = v[4 * k + 3];
        } else {
            w.x = v[2 * k]; w.y = v[2 * k + 1];
        }
        q[k] = w;
    }
}

template <typename T, int N>
__device__ inline void fill(T (&v)[N], T a) {
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = a;
}
// Value of lane + D (D > 0) or lane - D (D < 0) within the lane's row of 16
// (data-parallel primitive move, a vector ALU operation; 0 when that lane is
// outside the row).  For segments of K <= 16 lanes aligned to K.
template <int D>
__device__ inline int dpp_row_shift(int v) {
    static_assert(D != 0 && D > -16 && D < 16, "row shift");
    constexpr int ctrl = D > 0 ? 0x100 + D : 0x110 - D;  // row_shl:D / row_shr:-D
    return __builtin_amdgcn_update_dpp(0, v, ctrl, 0xf, 0xf, true);
}
template <int D, typename T>
__device__ inline T row_shift(T v) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, dpp_row_shift<D>(__builtin_bit_cast(int, v)));
    } else {
        const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
        const unsigned lo = (unsigned)dpp_row_shift<D>((int)(unsigned)u);
        const unsigned hi = (unsigned)dpp_row_shift<D>((int)(unsigned)(u >> 32));
        return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
    }
}

// One step of parallel cyclic reduction on the chunk-end rows
// (A x_{k-st} + B x_k + C x_{k+st} = R), neighbours from lanes k -+ st.
template <typename T>
__device__ inline void pcr_combine(int k, int K, int st, T& A, T& B, T& C, T& R, T Am, T Bm, T Cm, T Rm, T Ap, T Bp,
                                   T Cp, T Rp) {
    T nA = T(0), nB = B, nC = T(0), nR = R;
    if (k - st >= 0) {
        const T al = -A * line_rcp(Bm);
        nA = al * Am;
        nB += al * Cm;
        nR += al * Rm;
    }
    if (k + st < K) {
        const T ga = -C * line_rcp(Bp);
        nC = ga * Cp;
        nB += ga * Ap;
        nR += ga * Rp;
    }
    A = nA;
    B = nB;
    C = nC;
    R = nR;
}
template <int ST, typename T>
__device__ inline void pcr_step_dpp(int k, int K, T& A, T& B, T& C, T& R) {
    const T Am = row_shift<-ST>(A), Bm = row_shift<-ST>(B), Cm = row_shift<-ST>(C), Rm = row_shift<-ST>(R);
    const T Ap = row_shift<ST>(A), Bp = row_shift<ST>(B), Cp = row_shift<ST>(C), Rp = row_shift<ST>(R);
    pcr_combine(k, K, ST, A, B, C, R, Am, Bm, Cm, Rm, Ap, Bp, Cp, Rp);
}

// Tridiagonal systems A_k X_{k-1} + B_k X_k + C_k X_{k+1} = R_k, k = 0 ..
// K-1, one row per thread, each system on K consecutive threads of the
// workgroup (K a power of two, segments aligned to K; A_0 and C_{K-1} unused).
// K <= 64: parallel cyclic reduction with shuffles inside the segment, no
// barrier.  K > 64: cyclic reduction in LDS (each level keeps every other
// remaining row, one barrier per level) down to 64 rows, parallel cyclic
// reduction of those by the segment's first wavefront, then back substitution
// level by level.  Returns X_k and X_{k-1} (0 for k = 0).  Every thread of the
// workgroup calls it with the same K; sA, sB, sC, sR, sX: one element per
// thread.
template <typename T>
__device__ void seg_tridiag(int t, int k, int K, T A, T B, T C, T R, T* sA, T* sB, T* sC, T* sR, T* sX, T& X,
                            T& Xp) {
    const int lane = threadIdx.x & 63;
    auto wave_pcr = [&](int kk, int KK, T& a, T& b, T& c, T& r) {
        for (int st = 1; st < KK; st <<= 1) {
            const T Am = __shfl(a, lane - st, 64), Bm = __shfl(b, lane - st, 64);
            const T Cm = __shfl(c, lane - st, 64), Rm = __shfl(r, lane - st, 64);
            const T Ap = __shfl(a, lane + st, 64), Bp = __shfl(b, lane + st, 64);
            const T Cp = __shfl(c, lane + st, 64), Rp = __shfl(r, lane + st, 64);
            T nA = T(0), nB = b, nC = T(0), nR = r;
            if (kk - st >= 0) {
                const T al = -a * line_rcp(Bm);
                nA = al * Am;
                nB += al * Cm;
                nR += al * Rm;
            }
            if (kk + st < KK) {
                const T ga = -c * line_rcp(Bp);
                nC = ga * Cp;
                nB += ga * Ap;
                nR += ga * Rp;
            }
            a = nA;
            b = nB;
            c = nC;
            r = nR;
        }
    };
    if (K <= 64) {
        wave_pcr(k, K, A, B, C, R);
        X = R * line_rcp(B);
        Xp = __shfl(X, lane - 1, 64);
        if (k == 0) Xp = T(0);
        return;
    }
    sA[t] = A;
    sB[t] = B;
    sC[t] = C;
    sR[t] = R;
    __syncthreads();
    // reduction: at stride s the rows with (k + 1) % 2s == 0 absorb rows k -+ s
    // (which stop changing at that level)
    int s = 1;
    for (; K / s > 64; s <<= 1) {
        if (((k + 1) & (2 * s - 1)) == 0) {
            const int m = t - s;
            const T a = sA[t], c = sC[t];
            const T al = -a * line_rcp(sB[m]);
            T nA = al * sA[m], nB = sB[t] + al * sC[m], nC = T(0), nR = sR[t] + al * sR[m];
            if (k + s < K) {
                const int p = t + s;
                const T ga = -c * line_rcp(sB[p]);
                nC = ga * sC[p];
                nB += ga * sA[p];
                nR += ga * sR[p];
            }
            sA[t] = nA;
            sB[t] = nB;
            sC[t] = nC;
            sR[t] = nR;
        }
        __syncthreads();
    }
    // the 64 remaining rows (k = s (j + 1) - 1) on the segment's first wavefront
    const int base = t - k;
    if (k < 64) {
        const int kk = base + s * (k + 1) - 1;
        T a = sA[kk], b = sB[kk], c = sC[kk], r = sR[kk];
        wave_pcr(k, 64, a, b, c, r);
        sX[kk] = r * line_rcp(b);
    }
    __syncthreads();
    for (s >>= 1; s >= 1; s >>= 1) {
        if (((k + 1) & (2 * s - 1)) == s) {
            T v = sR[t];
            if (k >= s) v -= sA[t] * sX[t - s];
            if (k + s < K) v -= sC[t] * sX[t + s];
            sX[t] = v * line_rcp(sB[t]);
        }
        __syncthreads();
    }
    X = sX[t];
    Xp = k > 0 ? sX[t - 1] : T(0);
}

// Lanes per line for a line of `na` cells with at most LM cells per lane
// (power of two, <= 64).
template <int LM>
__device__ inline int wave_line_lanes(int na) {
    int K = 1;
    while (K * LM < na) K <<= 1;
    return K;
}

// One zebra half-sweep of line Gauss-Seidel: every line of parity `par`
// (lines par, par + 2, ...) among `nlines` lines of `na` cells is solved
// exactly,
//   (m + sum W) x - W_prev x_prev - W_next x_next = b + W_c- x_c- + W_c+ x_c+,
// the cross couplings W_c taken with the neighbour lines' current x (ZERO:
// with x = 0).  Cell (line, pos) sits at index line * sl + pos * sa of every
// array; Wa[c] couples cell c to the next cell along its line, Wc[c] to the
// same position on the next line (both zero past the last cell / line).
//
// A line is split into K chunks of L <= LM cells, one chunk per lane of a
// K-lane segment of a wavefront.  Each lane eliminates its chunk interior
// (Thomas with three right-hand sides) so that every interior unknown is
// y + u X_{k-1} + v X_k in the chunk-end unknowns X; the K chunk-end rows form
// a tridiagonal system solved by parallel cyclic reduction across the lanes
// (shuffles; with DPP, binary32 segments of at most 16 lanes use row shifts,
// measured faster for rows read from global memory and slower from LDS);
// back-substitution finishes.  Wave `wave` of `nwaves` takes lines
// wave * 64/K + ..., the next pass nwaves * 64/K lines further.  Needs na <=
// 64 LM.  The caller separates half-sweeps with a barrier.  I: index type
// (int where every index fits, as in LDS).  FULL: na == K LM (every chunk
// whole), the chunk bounds known at compile time.
template <typename T, int LM, bool ZERO, bool BF = true, bool DPP = false, typename I = long long, bool FULL = false>
__device__ void wave_line_sweep(int na, int nlines, int par, I sa, I sl, const T* __restrict__ m,
                                const T* __restrict__ Wa, const T* __restrict__ Wc, const T* __restrict__ b,
                                T* __restrict__ x, int wave, int nwaves) {
    const int nl = (nlines - par + 1) / 2;
    if (nl <= 0) return;
    const int K = wave_line_lanes<LM>(na);
    const int L = FULL ? LM : max(2, (na + K - 1) / K);
    const int lpw = 64 / K;
    const int lane = threadIdx.x & 63;
    const int k = lane & (K - 1);
    const int s0 = k * L;
    for (int q0 = wave * lpw; q0 < nl; q0 += nwaves * lpw) {
        const int ql = q0 + lane / K;
        const bool active = ql < nl;
        const int line = 2 * ql + par;
        const I lb = (I)(active ? line : 0) * sl;
        T vm[LM], va[LM], vcn[LM], vcs[LM], vb[LM], vxn[LM], vxs[LM];
        const T wprev = (active && s0 > 0 && (FULL || s0 - 1 < na)) ? Wa[lb + (I)(s0 - 1) * sa] : T(0);
        // a full chunk along a contiguous row, 16-byte aligned in every array
        // (the arrays share their element offsets): vector loads
        constexpr int VW = 16 / sizeof(T);
        const bool vec = sa == 1 && active && L == LM && s0 + LM <= na && (sl % VW) == 0 &&
                         ((reinterpret_cast<uintptr_t>(m + lb + s0) | reinterpret_cast<uintptr_t>(Wa + lb + s0) |
                           reinterpret_cast<uintptr_t>(Wc + lb + s0) | reinterpret_cast<uintptr_t>(b + lb + s0) |
                           reinterpret_cast<uintptr_t>(x + lb + s0)) & 15) == 0;
        if (vec) {
            const I c0 = lb + s0;
            load_vec<T, LM>(m + c0, vm);
            load_vec<T, LM>(Wa + c0, va);
            load_vec<T, LM>(Wc + c0, vcn);
            load_vec<T, LM>(b + c0, vb);
            if (line > 0) load_vec<T, LM>(Wc + c0 - sl, vcs);
            else fill<T, LM>(vcs, T(0));
            if (!ZERO && line + 1 < nlines) load_vec<T, LM>(x + c0 + sl, vxn);
            else fill<T, LM>(vxn, T(0));
            if (!ZERO && line > 0) load_vec<T, LM>(x + c0 - sl, vxs);
            else fill<T, LM>(vxs, T(0));
        } else if (!BF) {
#pragma unroll
            for (int q = 0; q < LM; ++q) {
                const int g = s0 + q;
                const bool ok = FULL ? active : (active && q < L && g < na);
                const I c = lb + (I)g * sa;
                vm[q] = ok ? m[c] : T(1);
                va[q] = ok ? Wa[c] : T(0);
                vcn[q] = ok ? Wc[c] : T(0);
                vcs[q] = (ok && line > 0) ? Wc[c - sl] : T(0);
                vb[q] = ok ? b[c] : T(0);
                vxn[q] = (!ZERO && ok && line + 1 < nlines) ? x[c + sl] : T(0);
                vxs[q] = (!ZERO && ok && line > 0) ? x[c - sl] : T(0);
            }
        } else {
            // branch-free (BF): every load reads a valid cell (indices clamped
            // into the line and the grid) and the value is masked afterwards,
            // so the loads issue back to back instead of one guarded block
            // each (much faster from LDS; measured slower for binary32 rows in
            // global memory, where guarded loads skip traffic).  A lane past
            // the last line reads line 0 (lb = 0) with no neighbour offsets:
            // line 0 minus sl would lie before the array.
            const I dn = (active && line + 1 < nlines) ? sl : 0, ds = (active && line > 0) ? -sl : 0;
#pragma unroll
            for (int q = 0; q < LM; ++q) {
                const int g = s0 + q;
                const bool ok = FULL ? active : (active && q < L && g < na);
                const I c = lb + (I)(FULL ? g : min(g, na - 1)) * sa;
                const T m_ = m[c], wa_ = Wa[c], wc_ = Wc[c], ws_ = Wc[c + ds], b_ = b[c];
                vm[q] = ok ? m_ : T(1);
                va[q] = ok ? wa_ : T(0);
                vcn[q] = ok ? wc_ : T(0);
                vcs[q] = (ok && ds != 0) ? ws_ : T(0);
                vb[q] = ok ? b_ : T(0);
                if (!ZERO) {
                    const T xn_ = x[c + dn], xs_ = x[c + ds];
                    vxn[q] = (ok && dn != 0) ? xn_ : T(0);
                    vxs[q] = (ok && ds != 0) ? xs_ : T(0);
                } else {
                    vxn[q] = vxs[q] = T(0);
                }
            }
        }
        T vd[LM], vr[LM];
#pragma unroll
        for (int q = 0; q < LM; ++q) {
            const T wp = (q == 0) ? wprev : va[q > 0 ? q - 1 : 0];
            vd[q] = vm[q] + ((wp + va[q]) + (vcs[q] + vcn[q]));
            vr[q] = vb[q] + vcn[q] * vxn[q] + vcs[q] * vxs[q];
        }
        auto coef = [&](int q, T& a, T& d, T& c, T& r) {
            a = -((q == 0) ? wprev : va[q > 0 ? q - 1 : 0]);
            d = vd[q];
            c = -va[q];
            r = vr[q];
        };
        T cp[LM], gy[LM], gu[LM], gv[LM];
#pragma unroll
        for (int q = 0; q < LM - 1; ++q) {
            if (q < L - 1) {
                T a, d, c, r;
                coef(q, a, d, c, r);
                const T den = (q == 0) ? d : d - a * cp[q > 0 ? q - 1 : 0];
                const T inv = line_rcp(den);
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
        // the next chunk's first row, y + u X_k + v X_{k+1} (binary64 row
        // shifts would need twice the moves and registers)
        const bool has_next = k + 1 < K;
        const bool rows16 = DPP && sizeof(T) == 4 && K <= 16;
        T yn, un, vn;
        if (rows16) {
            yn = row_shift<1>(gy[0]);
            un = row_shift<1>(gu[0]);
            vn = row_shift<1>(gv[0]);
        } else {
            yn = __shfl(gy[0], lane + 1, 64);
            un = __shfl(gu[0], lane + 1, 64);
            vn = __shfl(gv[0], lane + 1, 64);
        }
        if (!has_next) yn = un = vn = T(0);
        T A = aE * ul, B = dE + aE * vl + cE * un, C = cE * vn, R = rE - aE * yl - cE * yn;
        if (rows16) {
            if (K > 1) pcr_step_dpp<1>(k, K, A, B, C, R);
            if (K > 2) pcr_step_dpp<2>(k, K, A, B, C, R);
            if (K > 4) pcr_step_dpp<4>(k, K, A, B, C, R);
            if (K > 8) pcr_step_dpp<8>(k, K, A, B, C, R);
        } else {
            for (int st = 1; st < K; st <<= 1) {
                const T Am = __shfl(A, lane - st, 64), Bm = __shfl(B, lane - st, 64);
                const T Cm = __shfl(C, lane - st, 64), Rm = __shfl(R, lane - st, 64);
                const T Ap = __shfl(A, lane + st, 64), Bp = __shfl(B, lane + st, 64);
                const T Cp = __shfl(C, lane + st, 64), Rp = __shfl(R, lane + st, 64);
                pcr_combine(k, K, st, A, B, C, R, Am, Bm, Cm, Rm, Ap, Bp, Cp, Rp);
            }
        }
        const T X = R * line_rcp(B);
        T Xp = rows16 ? row_shift<-1>(X) : __shfl(X, lane - 1, 64);
        if (k == 0) Xp = T(0);
        if (active) {
#pragma unroll
            for (int q = 0; q < LM; ++q) {
                const int g = s0 + q;
                if (FULL || (q < L && g < na)) {
                    const T v = (q == L - 1) ? X
                                             : gy[q < LM - 1 ? q : 0] + gu[q < LM - 1 ? q : 0] * Xp +
                                                   gv[q < LM - 1 ? q : 0] * X;
                    x[lb + (I)g * sa] = v;
                }
            }
        }
    }
}

}  // namespace fld
