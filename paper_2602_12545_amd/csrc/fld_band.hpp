// Band-fused zebra line sweeps: both half-sweeps of one direction in one
// launch.
//
// A workgroup owns a band of R consecutive rows (R even) of the layout being
// swept.  Zebra line Gauss-Seidel solves first every row of parity p1, then
// every row of parity p2 = 1 - p1 from the fresh p1 rows.  A p2 row of the
// band needs the p1 rows just above and below it; the one outside the band
// (row r0 - 1 when p1 = 1, row r0 + R when p1 = 0) is solved here as well,
// from the same inputs and with the same arithmetic as in the band that owns
// it, so it is bit-identical to that band's value and the launch equals the
// two separate half-sweeps exactly.  Solved rows stay in LDS; the band's rows
// are written once at the end, in the same layout or transposed (so the next
// sweep direction reads rows again), optionally with the right-hand side
// transposed alongside.
//
// Inside a pass, a row of na cells is split into K chunks of L <= LM cells
// (the chunking of the one-half-sweep kernel), one chunk per thread; the
// chunk interior is eliminated locally and the K chunk-end unknowns are solved
// by parallel cyclic reduction with wavefront shuffles when K <= 64, else by
// seg_tridiag (cyclic reduction in LDS down to one wavefront's worth).
// (Longer chunks that keep 1024-cell rows inside one wavefront were measured
// slower: the per-lane Thomas chain doubles and occupancy halves.)
#pragma once

#include "fld_mg.hpp"

namespace fld {

constexpr int kBandWG = 512;

// LDS bytes of one k_band launch: R + 2 row slots (+ R rows of b when the
// right-hand side is transposed alongside), the cyclic-reduction arrays and
// the reduction scratch.
template <typename T>
inline size_t band_lds_bytes(int na, int R, bool with_b) {
    return sizeof(T) * ((size_t)(R + 2) * na + (with_b ? (size_t)R * na : 0) + 7 * (size_t)kBandWG) +
           16 * sizeof(double);
}

// A Krylov-accelerated level's vector updates folded into its sweeps
// (v == nullptr: none).  LINE_ZERO: the right-hand side is taken as
// b - s1 v (the level's second pass; v = A c1), and the band's rows of it are
// also stored, untransposed, in bout2 for the pass's later kernels.
// LINE_PROLONG: the coarse correction read from the level below is taken as
// f1 v + f2 ec (v = that level's c1: its two-step combination).  The
// coefficients come from the stage's G workgroup partials (part != nullptr,
// summed by every workgroup in the same order; the stage-0 fold's workgroup 0
// records rho1, s1 for stage 1) or from ks.
template <typename T>
struct BandKL {
    const T* v = nullptr;
    const double* part = nullptr;
    int G = 0;
    KLScal* ks = nullptr;
    T* bout2 = nullptr;
    int single = 0;
};

template <typename T, int LM, int MODE, int FIRST, bool OUT_T, bool WRITE_BT, bool DOT>
__global__ __launch_bounds__(kBandWG) void k_band(int nx, int ny, int R, int K, int L, const T* __restrict__ m,
                                                  const T* __restrict__ We, const T* __restrict__ Wn,
                                                  const T* __restrict__ b, const T* __restrict__ xin,
                                                  const T* __restrict__ ec, int nxc, T* __restrict__ xout,
                                                  T* __restrict__ bout, double* part, const Scalars* sc, int* ran,
                                                  BandKL<T> kl) {
    if (sc->done) return;
    if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
    extern __shared__ __align__(16) unsigned char band_smem[];
    constexpr int NT = kBandWG;
    T* rows = reinterpret_cast<T*>(band_smem);               // (R + 2) x nx: slot = row - (r0 - 1)
    T* bb = rows + (size_t)(R + 2) * nx;                      // R x nx (WRITE_BT)
    T* pcr = bb + (WRITE_BT ? (size_t)R * nx : 0);            // 7 x NT
    double* sh = reinterpret_cast<double*>(pcr + 7 * NT);
    T *sA = pcr, *sB = pcr + NT, *sC = pcr + 2 * NT, *sR = pcr + 3 * NT;
    T *sy0 = pcr + 4 * NT, *su0 = pcr + 5 * NT, *sv0 = pcr + 6 * NT;
    const int t = threadIdx.x, r0 = xcd_block(blockIdx.x, gridDim.x) * R;
    const int rend = min(r0 + R, ny);  // band rows [r0, rend)
    const int k = t % K, lpp = NT / K, s0 = k * L;
    const int lane = t & 63;
    const bool wave_pcr = K <= 64;
    double acc = 0.0;  // DOT: b.x over the band's rows, accumulated as they are solved
    // Krylov-level folds: s1 (LINE_ZERO), f1 and f2 (LINE_PROLONG)
    const bool fold_b = MODE == LINE_ZERO && kl.v != nullptr;
    const bool fold_e = MODE == LINE_PROLONG && kl.v != nullptr;
    T ks1 = T(0), kf1 = T(0), kf2 = T(1);
    if (fold_b || fold_e) {
        KLScal kk = *kl.ks;
        if (kl.part) {
            double v[3];
            if (fold_b) {
                kl_sum<0, NT>(kl.part, kl.G, v, sh);
                kl_coeffs<0>(v, kk, 0);
                if (blockIdx.x == 0 && t == 0) {
                    kl.ks->rho1 = kk.rho1;
                    kl.ks->s1 = kk.s1;
                }
            } else {
                kl_sum<1, NT>(kl.part, kl.G, v, sh);
                kl_coeffs<1>(v, kk, kl.single);
            }
        }
        ks1 = (T)kk.s1;
        kf1 = (T)kk.f1;
        kf2 = (T)kk.f2;
    }

    // Coefficients, right-hand side and (first parity) neighbour-row x of one
    // chunk of one row, loaded ahead of the solve, for rows that split into
    // whole aligned vector chunks (every lane's chunk is LM cells at a
    // 16-byte boundary).  Every address is valid (rows off the grid clamped
    // to the row itself); the solve masks what does not exist, so no load
    // waits for another.
    struct Coef {
        T vm[LM], vwe[LM], vwn[LM], vws[LM], vb[LM], xn[LM], xs[LM];
        T wwest;
    };
    auto load_coef_vec = [&](int row, Coef& C, bool with_x) {
        const size_t rb = (size_t)row * nx;
        const size_t rs = row > 0 ? rb - nx : rb, rn = row + 1 < ny ? rb + nx : rb;
        C.wwest = We[rb + (s0 > 0 ? s0 - 1 : 0)];
        load_vec<T, LM>(m + rb + s0, C.vm);
        load_vec<T, LM>(We + rb + s0, C.vwe);
        load_vec<T, LM>(Wn + rb + s0, C.vwn);
        load_vec<T, LM>(b + rb + s0, C.vb);
        if (fold_b) {
            T vv[LM];
            load_vec<T, LM>(kl.v + rb + s0, vv);
#pragma unroll
            for (int q = 0; q < LM; ++q) C.vb[q] -= ks1 * vv[q];
        }
        load_vec<T, LM>(Wn + rs + s0, C.vws);
        if (with_x && MODE != LINE_ZERO) {
            load_vec<T, LM>(xin + rn + s0, C.xn);
            load_vec<T, LM>(xin + rs + s0, C.xs);
            if (MODE == LINE_PROLONG) {
                // coarse correction of cells s0 .. s0 + LM - 1: LM / 2 values
                T en[LM / 2], es[LM / 2];
                const int ic = s0 >> 1;
                const size_t on = (size_t)((row + 1 < ny ? row + 1 : row) >> 1) * nxc + ic;
                const size_t os = (size_t)((row > 0 ? row - 1 : row) >> 1) * nxc + ic;
                load_vec<T, LM / 2>(ec + on, en);
                load_vec<T, LM / 2>(ec + os, es);
                if (fold_e) {
                    T cn[LM / 2], cs[LM / 2];
                    load_vec<T, LM / 2>(kl.v + on, cn);
                    load_vec<T, LM / 2>(kl.v + os, cs);
#pragma unroll
                    for (int q = 0; q < LM / 2; ++q) {
                        en[q] = kf1 * cn[q] + kf2 * en[q];
                        es[q] = kf1 * cs[q] + kf2 * es[q];
                    }
                }
#pragma unroll
                for (int q = 0; q < LM; ++q) {
                    C.xn[q] += en[q >> 1];
                    C.xs[q] += es[q >> 1];
                }
            }
        }
    };

    // Solve one row (or none, !active) of a pass; PH = 1: first parity
    // (neighbours from xin), PH = 2: second parity (neighbours from LDS).
    // The coefficients come from `pre` (PRE) or are loaded here.  Every
    // thread of the workgroup calls it (the LDS reduction has barriers).
    auto solve_row = [&](int row, bool active, const Coef* pre, auto pre_tag, auto full_tag, int PH) {
        constexpr bool PRE = decltype(pre_tag)::value;
        // FULL (always with PRE): the row splits into whole LM-cell chunks, so
        // the chunk bounds are compile-time constants
        constexpr bool FULL = PRE || decltype(full_tag)::value;
        const int Lc = FULL ? LM : L;
        // a wavefront whose rows are all idle skips the solve and leaves its
        // SIMD to the busy ones; with rows spanning wavefronts it still passes
        // the same barriers (the exchange, seg_tridiag's on identity rows,
        // the LDS reuse)
        if (!__any(active)) {
            if constexpr (LM == kLineMaxL) {
                if (!wave_pcr) {
                    __syncthreads();
                    T X, Xp;
                    seg_tridiag<T>(t, k, K, T(0), T(1), T(0), T(0), sA, sB, sC, sR, sy0, X, Xp);
                    __syncthreads();
                }
            }
            return;
        }
        const size_t rb = (size_t)row * nx;
        T vm[LM], vwe[LM], vwn[LM], vws[LM], vb[LM];
        T wwest;
        if constexpr (PRE) {
#pragma unroll
            for (int q = 0; q < LM; ++q) {
                vm[q] = pre->vm[q];
                vwe[q] = pre->vwe[q];
                vwn[q] = pre->vwn[q];
                vws[q] = row > 0 ? pre->vws[q] : T(0);
                vb[q] = pre->vb[q];
            }
            wwest = s0 > 0 ? pre->wwest : T(0);
        } else {
            wwest = (active && s0 > 0 && s0 - 1 < nx) ? We[rb + s0 - 1] : T(0);
            constexpr int VW = 16 / sizeof(T);
            const bool vec = active && L == LM && s0 + LM <= nx && ((rb + s0) % VW) == 0 && (nx % VW) == 0;
            if (vec) {
                load_vec<T, LM>(m + rb + s0, vm);
                load_vec<T, LM>(We + rb + s0, vwe);
                load_vec<T, LM>(Wn + rb + s0, vwn);
                load_vec<T, LM>(b + rb + s0, vb);
                if (fold_b) {
                    T vv[LM];
                    load_vec<T, LM>(kl.v + rb + s0, vv);
#pragma unroll
                    for (int q = 0; q < LM; ++q) vb[q] -= ks1 * vv[q];
                }
                if (row > 0) load_vec<T, LM>(Wn + rb + s0 - nx, vws);
                else fill<T, LM>(vws, T(0));
            } else {
#pragma unroll
                for (int q = 0; q < LM; ++q) {
                    const int g = s0 + q;
                    const bool ok = active && (FULL || (q < Lc && g < nx));
                    const size_t c = rb + g;
                    vm[q] = ok ? m[c] : T(1);
                    vwe[q] = ok ? We[c] : T(0);
                    vwn[q] = ok ? Wn[c] : T(0);
                    vws[q] = (ok && row > 0) ? Wn[c - nx] : T(0);
                    vb[q] = ok ? (fold_b ? b[c] - ks1 * kl.v[c] : b[c]) : T(0);
                }
            }
        }
        T vxn[LM], vxs[LM];
        // neighbour rows (whole chunks of the second parity: 16-byte LDS reads)
        if (FULL && PH == 2) {
            if (active && row + 1 < ny) load_vec<T, LM>(rows + (size_t)(row + 1 - (r0 - 1)) * nx + s0, vxn);
            else fill<T, LM>(vxn, T(0));
            if (active && row > 0) load_vec<T, LM>(rows + (size_t)(row - 1 - (r0 - 1)) * nx + s0, vxs);
            else fill<T, LM>(vxs, T(0));
        } else {
#pragma unroll
        for (int q = 0; q < LM; ++q) {
            const int g = s0 + q;
            const bool ok = active && (FULL || (q < Lc && g < nx));
            T xn = T(0), xs = T(0);
            if (ok) {
                if (PH == 2) {
                    if (row + 1 < ny) xn = rows[(size_t)(row + 1 - (r0 - 1)) * nx + g];
                    if (row > 0) xs = rows[(size_t)(row - 1 - (r0 - 1)) * nx + g];
                } else if (PRE) {
                    if (MODE != LINE_ZERO) {
                        if (row + 1 < ny) xn = pre->xn[q];
                        if (row > 0) xs = pre->xs[q];
                    }
                } else if (MODE != LINE_ZERO) {
                    if (row + 1 < ny) {
                        xn = xin[rb + nx + g];
                        if (MODE == LINE_PROLONG) {
                            const size_t ce = (size_t)((row + 1) >> 1) * nxc + (g >> 1);
                            xn += fold_e ? kf1 * kl.v[ce] + kf2 * ec[ce] : ec[ce];
                        }
                    }
                    if (row > 0) {
                        xs = xin[rb - nx + g];
                        if (MODE == LINE_PROLONG) {
                            const size_t ce = (size_t)((row - 1) >> 1) * nxc + (g >> 1);
                            xs += fold_e ? kf1 * kl.v[ce] + kf2 * ec[ce] : ec[ce];
                        }
                    }
                }
            }
            vxn[q] = xn;
            vxs[q] = xs;
        }
        }
        if (WRITE_BT && active && row >= r0 && row < rend) {
            if (FULL) {
                store_vec<T, LM>(bb + (size_t)(row - r0) * nx + s0, vb);
            } else {
#pragma unroll
                for (int q = 0; q < LM; ++q)
                    if (q < Lc && s0 + q < nx) bb[(size_t)(row - r0) * nx + s0 + q] = vb[q];
            }
        }
        // diagonal and right-hand side of every chunk row (the loaded
        // arrays die here, which keeps register pressure low)
        T vd[LM], vr[LM];
#pragma unroll
        for (int q = 0; q < LM; ++q) {
            const T ww = (q == 0) ? wwest : vwe[q > 0 ? q - 1 : 0];
            vd[q] = vm[q] + ((ww + vwe[q]) + (vws[q] + vwn[q]));
            vr[q] = vb[q] + vwn[q] * vxn[q] + vws[q] * vxs[q];
        }
        auto coef = [&](int q, T& a, T& d, T& c, T& r) {
            a = -((q == 0) ? wwest : vwe[q > 0 ? q - 1 : 0]);
            d = vd[q];
            c = -vwe[q];
            r = vr[q];
        };
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
#pragma unroll
        for (int q = LM - 3; q >= 0; --q) {
            if (q < Lc - 2) {
                gy[q] -= cp[q] * gy[q + 1];
                gu[q] -= cp[q] * gu[q + 1];
                gv[q] -= cp[q] * gv[q + 1];
            }
        }
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
        const bool has_next = k + 1 < K;
        T X, Xp;
        if (LM > kLineMaxL || wave_pcr) {
            T yn = __shfl(gy[0], lane + 1, 64), un = __shfl(gu[0], lane + 1, 64), vn = __shfl(gv[0], lane + 1, 64);
            if (!has_next) yn = un = vn = T(0);
            T A = aE * ul, B = dE + aE * vl + cE * un, C = cE * vn, Rr = rE - aE * yl - cE * yn;
            for (int st = 1; st < K; st <<= 1) {
                const T Am = __shfl(A, lane - st, 64), Bm = __shfl(B, lane - st, 64);
                const T Cm = __shfl(C, lane - st, 64), Rm = __shfl(Rr, lane - st, 64);
                const T Ap = __shfl(A, lane + st, 64), Bp = __shfl(B, lane + st, 64);
                const T Cp = __shfl(C, lane + st, 64), Rp = __shfl(Rr, lane + st, 64);
                T nA = T(0), nB = B, nC = T(0), nR = Rr;
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
                Rr = nR;
            }
            X = Rr * line_rcp(B);
            Xp = __shfl(X, lane - 1, 64);
            if (k == 0) Xp = T(0);
        } else if constexpr (LM == kLineMaxL) {
            sy0[t] = gy[0];
            su0[t] = gu[0];
            sv0[t] = gv[0];
            __syncthreads();
            const T yn = has_next ? sy0[t + 1] : T(0), un = has_next ? su0[t + 1] : T(0);
            const T vn = has_next ? sv0[t + 1] : T(0);
            // sy0 is free again once seg_tridiag's first barrier has passed
            seg_tridiag<T>(t, k, K, aE * ul, dE + aE * vl + cE * un, cE * vn, rE - aE * yl - cE * yn, sA, sB, sC,
                           sR, sy0, X, Xp);
        }
        if (active) {
            T* dst = rows + (size_t)(row - (r0 - 1)) * nx;
            const bool own = row >= r0 && row < rend;  // a band row, not the halo
            if (FULL) {
                T out[LM];
#pragma unroll
                for (int q = 0; q < LM; ++q) {
                    out[q] = (q == LM - 1) ? X
                                           : gy[q < LM - 1 ? q : 0] + gu[q < LM - 1 ? q : 0] * Xp +
                                                 gv[q < LM - 1 ? q : 0] * X;
                    if (DOT && own) acc += (double)vb[q] * (double)out[q];
                }
                store_vec<T, LM>(dst + s0, out);
            } else {
#pragma unroll
                for (int q = 0; q < LM; ++q) {
                    const int g = s0 + q;
                    if (q < Lc && g < nx) {
                        const T v = (q == Lc - 1) ? X
                                                 : gy[q < LM - 1 ? q : 0] + gu[q < LM - 1 ? q : 0] * Xp +
                                                       gv[q < LM - 1 ? q : 0] * X;
                        dst[g] = v;
                        if (DOT && own) acc += (double)vb[q] * (double)v;
                    }
                }
            }
        }
        if (LM == kLineMaxL && !wave_pcr) __syncthreads();  // the LDS reduction arrays are reused next pass
    };
    // `count` rows start, start + 2, ..., lpp rows per pass
    auto solve_rows = [&](int start, int count, int PH, auto full_tag) {
        for (int q0 = 0; q0 < count; q0 += lpp) {
            const int ql = q0 + t / K;
            const bool active = ql < count;
            const int row = start + 2 * (active ? ql : 0);
            solve_row(row, active, nullptr, std::false_type{}, full_tag, PH);
        }
    };

    constexpr int P1 = FIRST, P2 = 1 - FIRST;
    // first-parity rows in [r0 - 1, r0 + R], second-parity rows in [r0, rend)
    int s1 = r0 - 1;
    if (s1 < 0 || (s1 & 1) != P1) s1 += (s1 < 0) ? (P1 == 1 ? 2 : 1) : 1;
    const int e1 = min(r0 + R, ny - 1);
    const int n1 = s1 <= e1 ? (e1 - s1) / 2 + 1 : 0;
    const int s2 = ((r0 & 1) == P2) ? r0 : r0 + 1;
    const int n2 = s2 < rend ? (rend - 1 - s2) / 2 + 1 : 0;
    constexpr int VW = 16 / sizeof(T);
    const bool whole_vec =
        L == LM && K * LM == nx && (nx % VW) == 0 &&
        ((reinterpret_cast<uintptr_t>(m) | reinterpret_cast<uintptr_t>(We) | reinterpret_cast<uintptr_t>(Wn) |
          reinterpret_cast<uintptr_t>(b) | (MODE != LINE_ZERO ? reinterpret_cast<uintptr_t>(xin) : 0)) & 15) == 0 &&
        (MODE != LINE_PROLONG || ((nxc % VW) == 0 && (reinterpret_cast<uintptr_t>(ec) & 15) == 0 && LM / 2 >= VW)) &&
        (kl.v == nullptr || (reinterpret_cast<uintptr_t>(kl.v) & 15) == 0);
    if (sizeof(T) == 4 && whole_vec && n1 <= lpp && n2 <= lpp) {
        // one pass per parity: the second pass's coefficients are loaded
        // before the first pass is solved, so their latency overlaps it
        // (binary32 only: binary64 lacks the registers).  Idle row slots
        // solve a copy of the first row of their pass and store nothing.
        const int ql = t / K;
        const bool a1 = ql < n1, a2 = ql < n2;
        // (a parity with no row here loads band row r0, which exists)
        const int row1 = n1 > 0 ? s1 + 2 * (a1 ? ql : 0) : r0;
        const int row2 = n2 > 0 ? s2 + 2 * (a2 ? ql : 0) : r0;
        Coef C1, C2;
        if (__any(a1)) load_coef_vec(row1, C1, true);
        if (__any(a2)) load_coef_vec(row2, C2, false);
        solve_row(row1, a1, &C1, std::true_type{}, std::true_type{}, 1);
        __syncthreads();
        solve_row(row2, a2, &C2, std::true_type{}, std::true_type{}, 2);
    } else {
        if (L == LM && K * LM == nx) {
            solve_rows(s1, n1, 1, std::true_type{});
            __syncthreads();
            solve_rows(s2, n2, 2, std::true_type{});
        } else {
            solve_rows(s1, n1, 1, std::false_type{});
            __syncthreads();
            solve_rows(s2, n2, 2, std::false_type{});
        }
    }
    __syncthreads();
    // band rows out
    const int nr = rend - r0;
    if (!OUT_T) {
        for (int e = t; e < nr * nx; e += NT) {
            const int rr = e / nx, i = e - rr * nx;
            xout[(size_t)(r0 + rr) * nx + i] = rows[(size_t)(rr + 1) * nx + i];
        }
    } else {
        // transposed: column i of the band becomes nr consecutive values of row i
        for (int e = t; e < nr * nx; e += NT) {
            const int i = e / nr, rr = e - i * nr;
            xout[(size_t)i * ny + r0 + rr] = rows[(size_t)(rr + 1) * nx + i];
            if (WRITE_BT) bout[(size_t)i * ny + r0 + rr] = bb[(size_t)rr * nx + i];
        }
        if (WRITE_BT && fold_b && kl.bout2)
            for (int e = t; e < nr * nx; e += NT) {
                const int rr = e / nx, i = e - rr * nx;
                kl.bout2[(size_t)(r0 + rr) * nx + i] = bb[(size_t)rr * nx + i];
            }
    }
    if (DOT) {
        const double tot = block_sum(acc, sh);
        if (t == 0) part[blockIdx.x] = tot;
    }
}

}  // namespace fld
