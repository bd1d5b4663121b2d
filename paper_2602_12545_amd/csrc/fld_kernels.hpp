// HIP kernels of the implicit FLD radiation step (gfx950, wave64).
//
// Layout: cell arrays row-major [ny][nx].  The assembly runs one thread per
// cell on 64 x 4 workgroups and reads its neighbours' fields straight from
// global memory (the rows are shared through L2); 1D kernels stream with a
// grid-stride loop.  Reductions: wave64 butterfly (shfl_xor) + LDS per
// workgroup, one FP64 partial per workgroup, summed in a fixed order by the
// kernel that consumes them, so every reduction is deterministic.
#pragma once
#include "fld_internal.hpp"

namespace fld {

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------

__device__ inline int ltid() { return threadIdx.y * blockDim.x + threadIdx.x; }
__device__ inline int lsize() { return blockDim.x * blockDim.y; }

// Workgroup b of G, renumbered so that each XCD runs a contiguous range: the
// dispatcher deals workgroups to the 8 XCDs in turn (b -> XCD b mod 8), and
// neighbouring tiles then share that XCD's L2 (halo rows, partial lines of
// transposed writes).  A bijection of [0, G).
__device__ inline int xcd_block(int b, int G) {
    constexpr int X = 8;
    const int x = b % X, j = b / X, q = G / X, rem = G % X;
    return (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + j;
}

// Tile (tbx, tby) of a 2D grid of workgroups, in the XCD-aware order of
// xcd_block over the row-major workgroup numbering.
__device__ inline void xcd_tile(int& tbx, int& tby) {
    const int b = xcd_block(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    tbx = b % gridDim.x;
    tby = b / gridDim.x;
}

// Sum over the workgroup; the result is valid in thread 0.  sh: >= 16 doubles.
__device__ inline double block_sum(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int t = ltid();
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (t == 0) {
        const int nw = (lsize() + 63) >> 6;
        for (int w = 0; w < nw; ++w) r += sh[w];
    }
    __syncthreads();
    return r;
}

// Maximum over the workgroup; the result is valid in thread 0.
__device__ inline double block_max(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int t = ltid();
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    double r = 0.0;
    if (t == 0) {
        const int nw = (lsize() + 63) >> 6;
        for (int w = 0; w < nw; ++w) r = fmax(r, sh[w]);
    }
    __syncthreads();
    return r;
}

// Minimum over the workgroup; the result is valid in thread 0.
__device__ inline double block_min(double v, double* sh) {
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    const int t = ltid();
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    double r = INFINITY;
    if (t == 0) {
        const int nw = (lsize() + 63) >> 6;
        for (int w = 0; w < nw; ++w) r = fmin(r, sh[w]);
    }
    __syncthreads();
    return r;
}

__device__ inline unsigned nblocks2d() { return gridDim.x * gridDim.y; }
__device__ inline unsigned bid2d() { return blockIdx.y * gridDim.x + blockIdx.x; }

// ---------------------------------------------------------------------------
// flux limiters lambda(R) (Section 2: FLD closure and asymptotic limits)
// ---------------------------------------------------------------------------

__device__ inline double limiter(double R, int kind) {
    if (kind == LIM_DIFFUSION) return 1.0 / 3.0;
    if (kind == LIM_MINERBO) {
        return (R <= 1.5) ? 2.0 / (3.0 + sqrt(9.0 + 12.0 * R * R)) : 1.0 / (1.0 + R + sqrt(1.0 + 2.0 * R));
    }
    // Levermore-Pomraning (coth R - 1/R)/R.  Series below 0.1 (the closed form
    // cancels there); coth R = 1 + 2/expm1(2R) above.
    if (R < 0.1) {
        const double R2 = R * R;
        return 1.0 / 3.0 + R2 * (-1.0 / 45.0 + R2 * (2.0 / 945.0 + R2 * (-1.0 / 4725.0 + R2 * (2.0 / 93555.0))));
    }
    if (R > 20.0) return (1.0 - 1.0 / R) / R;
    return (1.0 + 2.0 / expm1(2.0 * R) - 1.0 / R) / R;
}

// Conductance dt dS D / h of an interior face between cell L and cell R.
// sigma_f: distance-weighted kappa_R rho of the two cells (harmonic mean of
// the diffusivities); E_f: linear interpolation to the face; R from the
// face-normal two-point gradient (Section 3.2.1 interface coefficient).
__device__ inline double face_W(double EL, double sL, double ER, double sR, double hL, double hR,
                                double dS, double dt, int lim) {
    const double h = hL + hR;
    const double sf = (hL * sL + hR * sR) / h;
    const double Ef = (hR * EL + hL * ER) / h;
    const double R = fabs(ER - EL) / (h * sf * Ef);
    const double D = kC * limiter(R, lim) / sf;
    return dt * dS * D / h;
}

// Boundary-face additions to the diagonal (bd) and right-hand side (br).
__device__ inline void boundary_face(int kind, double value, double Eg, double E1, double sig1, double h1,
                                     double dS, double dt, int lim, double& bd, double& br) {
    if (kind == BC_DIRICHLET_FACE) {
        const double Eb = kARad * value * value * value * value;
        const double R = fabs(Eb - E1) / (h1 * sig1 * Eb);
        const double W = dt * dS * (kC * limiter(R, lim) / sig1) / h1;
        bd += W;
        br += W * Eb;
    } else if (kind == BC_DIRICHLET_GHOST) {
        const double h = 2.0 * h1;
        const double Ef = 0.5 * (E1 + Eg);
        const double R = fabs(Eg - E1) / (h * sig1 * Ef);
        const double W = dt * dS * (kC * limiter(R, lim) / sig1) / h;
        bd += W;
        br += W * Eg;
    } else if (kind == BC_FLUX_IN) {
        br += dt * dS * value;
    } else if (kind == BC_FREE_STREAM) {
        bd += dt * dS * kC;
    } else if (kind == BC_MILNE) {
        // E_b = -2/(3 sigma) dE/dn with dE/dn = (E_b - E_1)/h1: E_b = a E_1/(1+a),
        // a = 2/(3 sigma h1); R = 3/2 on the face; outward flux D E_1/(h1 (1+a))
        const double a = 2.0 / (3.0 * sig1 * h1);
        bd += dt * dS * (kC * limiter(1.5, lim) / sig1) / (h1 * (1.0 + a));
    }
}

// ---------------------------------------------------------------------------
// metrics (Section 3.2.1: g = dS/dV, alpha from volume centres)
// ---------------------------------------------------------------------------

// Offset of the volume-weighted mean angle of [a, a + h] from a (weight sin th):
//   (sin a * int_0^h u cos u du + cos a * int_0^h u sin u du) / (cos a - cos(a + h)).
// int u sin u = sin h - h cos h is summed as its alternating series
// sum_k (-1)^(k+1) 2k h^(2k+1) / (2k+1)! for h < 0.3, where the closed form cancels.
__device__ inline double theta_offset(double a, double h) {
    const double sh = sin(0.5 * h);
    const double one_minus_cos = 2.0 * sh * sh;
    const double int_ucos = h * sin(h) - one_minus_cos;
    double int_usin;
    if (h < 0.3) {
        const double h2 = h * h;
        double term = h * h2 / 3.0, acc = 0.0;
        for (int k = 1; k <= 8; ++k) {
            acc += (k & 1) ? term : -term;
            term *= h2 / ((2.0 * k) * (2.0 * k + 3.0));
        }
        int_usin = acc;
    } else {
        int_usin = sin(h) - h * cos(h);
    }
    const double sa = sin(a), ca = cos(a);
    return (sa * int_ucos + ca * int_usin) / (sa * sin(h) + ca * one_minus_cos);
}

// Grid metrics from the face coordinates.  Spherical forms are arranged
// without cancellation for thin cells: r+^3 - r-^3 = dr (r+^2 + r+ r- + r-^2),
// volume-centre radius r_c = 3/4 (r+ + r-)(r+^2 + r-^2) / (r+^2 + r+ r- + r-^2)
// with r_c - r- = dr (6 r-^2 + 8 r- dr + 3 dr^2) / (4 (r+^2 + r+ r- + r-^2)),
// cos th- - cos th+ = 2 sin((th- + th+)/2) sin(dth/2).
static __global__ void k_metrics(int geom, int nx, int ny, const double* __restrict__ xf, const double* __restrict__ yf,
                          double* vx, double* vy, double* sx, double* sy, double* ax, double* hxL, double* hxR,
                          double* hyL, double* hyR, double* arc) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nx) {
        const double a = xf[t], b = xf[t + 1], d = b - a;
        if (geom == 0) {
            vx[t] = d;
            ax[t] = d;
            arc[t] = 1.0;
            hxR[t] = 0.5 * d;
            hxL[t + 1] = 0.5 * d;
        } else {
            const double q = b * b + a * b + a * a;
            vx[t] = d * q / 3.0;
            ax[t] = 0.5 * d * (a + b);
            arc[t] = 0.75 * (a + b) * (a * a + b * b) / q;
            const double off = d * (6.0 * a * a + 8.0 * a * d + 3.0 * d * d) / (4.0 * q);
            hxR[t] = off;
            hxL[t + 1] = d - off;
        }
    }
    if (t < ny) {
        const double a = yf[t], b = yf[t + 1], d = b - a;
        if (geom == 0) {
            vy[t] = d;
            hyR[t] = 0.5 * d;
            hyL[t + 1] = 0.5 * d;
        } else {
            vy[t] = 2.0 * sin(0.5 * (a + b)) * sin(0.5 * d);
            const double off = theta_offset(a, d);
            hyR[t] = off;
            hyL[t + 1] = d - off;
        }
    }
    if (t == 0) {
        hxL[0] = 0.0;
        hxR[nx] = 0.0;
        hyL[0] = 0.0;
        hyR[ny] = 0.0;
    }
    if (t <= nx) sx[t] = (geom == 0) ? 1.0 : xf[t] * xf[t];
    if (t <= ny) sy[t] = (geom == 0) ? 1.0 : sin(yf[t]);
}

// ---------------------------------------------------------------------------
// assembly (Section 3.2.1 coefficient list with T eliminated; steps 2-5)
// ---------------------------------------------------------------------------

struct AsmIn {
    const double *E, *T, *rho, *kR, *kP, *cv, *ghost;
    double dt;
    int lim;
    BCDev bc;
    const double *fx, *fy;  // face mass fluxes of the advection term ([ny][nx+1], [ny+1][nx]); null: none
    // E that the face coefficients D (interior and boundary) and the advection
    // term are evaluated from; null: E itself.  A sub-cycled step passes its
    // starting E^n here for every sub-step (Section 3.2.1 steps 1-2 once per step).
    const double* Eop;
};
struct AsmOut {
    double *We, *Wn, *m, *rhs, *s;
    int* err;
    double* part;   // per-workgroup partial maxima of the diagonal (k_reduce_max)
    double *bside, *rside;  // per boundary face (packed like the ghost array): that side's diagonal and
                            // right-hand-side terms, for the face fluxes (null: not kept)
};

// Assembly of one cell; returns its diagonal.
// One side's boundary face of a cell: its terms are added to the cell's and,
// when kept, recorded at slot k of the packed side arrays.
__device__ inline void side_face(int k, int kind, double value, double Eg, double E1, double sig1, double h1,
                                 double dS, double dt, int lim, const AsmOut& out, double& bd, double& br) {
    double d = 0.0, r = 0.0;
    boundary_face(kind, value, Eg, E1, sig1, h1, dS, dt, lim, d, r);
    bd += d;
    br += r;
    if (out.bside) {
        out.bside[k] = d;
        out.rside[k] = r;
    }
}

__device__ inline double assemble_cell(const Metrics& g, const AsmIn& in, const AsmOut& out, int i, int j) {
    const int nx = g.nx, ny = g.ny;
    const size_t c = (size_t)j * nx + i;
    const double* Eop = in.Eop ? in.Eop : in.E;
    const double E = in.E[c], Eo = Eop[c], T = in.T[c], rho = in.rho[c], kR = in.kR[c], kP = in.kP[c],
                 cv = in.cv[c];
    const bool ok = isfinite(E) && E > 0.0 && isfinite(Eo) && Eo > 0.0 && isfinite(T) && T > 0.0 &&
                    isfinite(rho) && rho > 0.0 && isfinite(kR) && kR > 0.0 && isfinite(kP) && kP >= 0.0 &&
                    isfinite(cv) && cv >= 0.0;
    if (!ok) atomicOr(out.err, 1);
    const double dt = in.dt;
    const int lim = in.lim;
    const double sig = kR * rho;
    const double vyj = g.vy[j], axi = g.ax[i], arci = g.arc[i];
    double bd = 0.0, br = 0.0, Ww = 0.0, We = 0.0, Ws = 0.0, Wn = 0.0;
    // x faces
    if (i > 0) {
        const size_t w = c - 1;
        Ww = face_W(Eop[w], in.kR[w] * in.rho[w], Eo, sig, g.hxL[i], g.hxR[i], g.sx[i] * vyj, dt, lim);
    } else {
        const double Eg = (in.bc.kind[0] == BC_DIRICHLET_GHOST) ? in.ghost[j] : 0.0;
        side_face(j, in.bc.kind[0], in.bc.value[0], Eg, Eo, sig, g.hxR[0], g.sx[0] * vyj, dt, lim, out, bd, br);
    }
    if (i + 1 < nx) {
        const size_t e = c + 1;
        We = face_W(Eo, sig, Eop[e], in.kR[e] * in.rho[e], g.hxL[i + 1], g.hxR[i + 1], g.sx[i + 1] * vyj, dt, lim);
    } else {
        const double Eg = (in.bc.kind[1] == BC_DIRICHLET_GHOST) ? in.ghost[ny + j] : 0.0;
        side_face(ny + j, in.bc.kind[1], in.bc.value[1], Eg, Eo, sig, g.hxL[nx], g.sx[nx] * vyj, dt, lim, out, bd,
                  br);
    }
    // y faces (theta distances are arc lengths at the volume-centre radius)
    if (j > 0) {
        const size_t s = c - nx;
        Ws = face_W(Eop[s], in.kR[s] * in.rho[s], Eo, sig, g.hyL[j] * arci, g.hyR[j] * arci, axi * g.sy[j], dt, lim);
    } else {
        const double Eg = (in.bc.kind[2] == BC_DIRICHLET_GHOST) ? in.ghost[2 * ny + i] : 0.0;
        side_face(2 * ny + i, in.bc.kind[2], in.bc.value[2], Eg, Eo, sig, g.hyR[0] * arci, axi * g.sy[0], dt, lim,
                  out, bd, br);
    }
    if (j + 1 < ny) {
        const size_t n = c + nx;
        Wn = face_W(Eo, sig, Eop[n], in.kR[n] * in.rho[n], g.hyL[j + 1] * arci, g.hyR[j + 1] * arci,
                    axi * g.sy[j + 1], dt, lim);
    } else {
        const double Eg = (in.bc.kind[3] == BC_DIRICHLET_GHOST) ? in.ghost[2 * ny + nx + i] : 0.0;
        side_face(2 * ny + nx + i, in.bc.kind[3], in.bc.value[3], Eg, Eo, sig, g.hyL[ny] * arci, axi * g.sy[ny], dt,
                  lim, out, bd, br);
    }
    // reflecting and axis sides carry no flux (boundary_face ignores them)
    // cell terms: C_V = rho c_v, beta = kappa_P rho c dt, X = 4 beta a_R T^3, f = C_V/(C_V+X)
    const double CV = rho * cv;
    const double beta = kP * rho * kC * dt;
    const double T3 = T * T * T;
    const double X = 4.0 * beta * kARad * T3;
    const double den = CV + X;
    const double f = den > 0.0 ? CV / den : 1.0;
    const double dV = g.vx[i] * vyj;
    const double mass = dV * (1.0 + beta * f);
    const double sumW = ((Ww + We) + Ws) + Wn;
    const double diag = mass + sumW + bd;
    // explicit advection (Section 3.2.1 advection term): dV S_adv = sum over
    // the faces of +-dS f e_r, e_r = E / rho of the upwind cell, the boundary
    // cell's own e_r outside the grid; added as dt dV S_adv
    double adv = 0.0;
    if (in.fx) {
        const size_t fc = (size_t)j * (nx + 1) + i;
        const double flo = in.fx[fc], fhi = in.fx[fc + 1], er = Eo / rho;
        const double erlo = i > 0 ? Eop[c - 1] / in.rho[c - 1] : er;
        const double erhi = i + 1 < nx ? Eop[c + 1] / in.rho[c + 1] : er;
        adv += g.sx[i] * vyj * flo * (flo >= 0.0 ? erlo : er) - g.sx[i + 1] * vyj * fhi * (fhi >= 0.0 ? er : erhi);
    }
    if (in.fy) {
        const double flo = in.fy[c], fhi = in.fy[c + nx], er = Eo / rho;
        const double erlo = j > 0 ? Eop[c - nx] / in.rho[c - nx] : er;
        const double erhi = j + 1 < ny ? Eop[c + nx] / in.rho[c + nx] : er;
        adv += axi * g.sy[j] * flo * (flo >= 0.0 ? erlo : er) - axi * g.sy[j + 1] * fhi * (fhi >= 0.0 ? er : erhi);
    }
    if (!isfinite(adv)) atomicOr(out.err, 1);
    out.We[c] = We;
    out.Wn[c] = Wn;
    out.m[c] = mass + bd;
    out.rhs[c] = (dV * (E + beta * f * kARad * T3 * T) + br) + dt * adv;
    out.s[c] = 1.0 / sqrt(diag);
    return diag;
}

// One thread per cell computes its four faces (each interior face is computed
// identically by its two cells, so the matrix is exactly symmetric), the
// boundary terms and the cell terms C_V, beta, f.
static __global__ __launch_bounds__(256) void k_assemble(Metrics g, AsmIn in, AsmOut out) {
    const int i = blockIdx.x * TBX + threadIdx.x;
    const int j = blockIdx.y * TBY + threadIdx.y;
    const int nx = g.nx, ny = g.ny;
    __shared__ double sh[16];
    const double diag = (i < nx && j < ny) ? assemble_cell(g, in, out, i, j) : 0.0;
    const double bm = block_max(diag, sh);
    if (ltid() == 0) out.part[bid2d()] = bm;
}

// Full diagonal and copies of the FP64 operator (test access).
static __global__ void k_get_operator(int nx, int ny, const double* We, const double* Wn, const double* m,
                               const double* rhs, double* oWe, double* oWn, double* odiag, double* orhs) {
    const int i = blockIdx.x * TBX + threadIdx.x;
    const int j = blockIdx.y * TBY + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const size_t c = (size_t)j * nx + i;
    if (oWe) oWe[c] = We[c];
    if (oWn) oWn[c] = Wn[c];
    if (orhs) orhs[c] = rhs[c];
    if (odiag) {
        const double ww = i > 0 ? We[c - 1] : 0.0;
        const double ws = j > 0 ? Wn[c - nx] : 0.0;
        odiag[c] = m[c] + (((ww + We[c]) + ws) + Wn[c]);
    }
}

// ---------------------------------------------------------------------------
// gas update (Section 3.2.1: psi_5, psi_6, psi_11)
// ---------------------------------------------------------------------------
static __global__ __launch_bounds__(256) void k_gas_update(int n, const double* __restrict__ E, const double* __restrict__ Tn,
                                                    const double* __restrict__ rho, const double* __restrict__ kP,
                                                    const double* __restrict__ cv, double dt, double* __restrict__ Tout) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
        const double T = Tn[c], r = rho[c];
        const double CV = r * cv[c];
        const double beta = kP[c] * r * kC * dt;
        const double T3 = T * T * T;
        const double X = 4.0 * beta * kARad * T3;
        Tout[c] = (CV * T + 3.0 * beta * kARad * T3 * T + beta * E[c]) / (CV + X);
    }
}

}  // namespace fld
