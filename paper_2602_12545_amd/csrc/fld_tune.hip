// Autotuner (fld_tune, fld_batch_tune, see include/fld.h): times candidate
// smoother schedules, multigrid depths, CG chunk lengths (single grid) and
// workgroup sizes / multigrid depths (batch) on the caller's own fields and
// returns the fastest configuration whose steps converge.  Built on the
// public entry points only; every trial runs on scratch copies of E and T.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include <hip/hip_runtime.h>

#include "fld.h"

namespace {

struct Scratch {
    double* E = nullptr;
    double* T = nullptr;
    ~Scratch() {
        if (E) (void)hipFree(E);
        if (T) (void)hipFree(T);
    }
};

// Mean wall time (ms) of `reps` steps after one untimed step; each step starts
// from the caller's E, T.  Returns the status and iterations of the last step.
template <class StepFn>
fld_status time_steps(StepFn step, const double* E0, const double* T0, Scratch& s, size_t n, hipStream_t st,
                      int reps, float* ms, int* iters) {
    fld_status last = FLD_OK;
    double tot = 0.0;
    for (int r = 0; r <= reps; ++r) {
        if (hipMemcpyAsync(s.E, E0, n * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(s.T, T0, n * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return FLD_EHIP;
        auto t0 = std::chrono::steady_clock::now();
        last = step(iters);
        if (hipStreamSynchronize(st) != hipSuccess) return FLD_EHIP;
        const double dt = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (r > 0) tot += dt;
        if (last != FLD_OK) break;
    }
    *ms = (float)(tot / std::max(1, reps));
    return last;
}

void record(fld_tune_entry* entries, int32_t max_entries, int32_t* n, const fld_options& o, int32_t threads,
            fld_status st, int iters, float ms) {
    if (entries && *n < max_entries) {
        fld_tune_entry& e = entries[*n];
        e.opt = o;
        e.threads = threads;
        e.status = st;
        e.inner_iters = iters;
        e.ms = ms;
    }
    ++*n;
}

}  // namespace

extern "C" {

fld_status fld_tune(const fld_grid* grid, const fld_options* base, const double* E, const double* T, const double* rho,
                    const double* kappa_R, const double* kappa_P, const double* c_v, const double* ghost_E, double dt,
                    int32_t reps, fld_options* best, fld_tune_entry* entries, int32_t max_entries,
                    int32_t* n_entries, void* stream) {
    if (!grid || !best || !E || !T || reps < 1 || grid->nx < 1 || grid->ny < 1) return FLD_EINVAL;
    fld_options b0;
    if (base) b0 = *base;
    else fld_default_options(&b0);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n = (size_t)grid->nx * grid->ny;
    Scratch s;
    if (hipMalloc(&s.E, n * sizeof(double)) != hipSuccess || hipMalloc(&s.T, n * sizeof(double)) != hipSuccess)
        return FLD_ENOMEM;
    // candidates: smoother schedule x coarsest-level size x CG chunk length
    // x multigrid cycle (line smoothers only: point smoothing has no LDS
    // sub-cycle, so the cycle does not change it)
    std::vector<fld_options> cand;
    const bool lines_fit = grid->nx <= 4096 && grid->ny <= 4096;
    for (int sm : {FLD_SMOOTH_LINE, FLD_SMOOTH_LINE_SPLIT, FLD_SMOOTH_POINT}) {
        if (sm != FLD_SMOOTH_POINT && !lines_fit) continue;
        for (int cy : {FLD_MG_CYCLE_K, FLD_MG_CYCLE_V, FLD_MG_CYCLE_W2, FLD_MG_CYCLE_KL_K, FLD_MG_CYCLE_KL_W2}) {
            if (sm == FLD_SMOOTH_POINT && cy != b0.mg_cycle) continue;
            for (int cm : {64, 256, 1024, 4096})
                for (int ch : {8, 16, 4}) {
                    fld_options o = b0;
                    o.smoother = sm;
                    o.mg_cycle = cy;
                    o.mg_coarse_max = cm;
                    o.chunk = ch;
                    o.use_graph = 1;
                    cand.push_back(o);
                }
        }
    }
    int32_t cnt = 0;
    float best_ms = INFINITY;
    fld_status overall = FLD_ENOCONV;
    for (const fld_options& o : cand) {
        fld_ctx* ctx = nullptr;
        fld_status cs = fld_create(&ctx, grid, &o, stream);
        if (cs != FLD_OK) {
            fld_destroy(ctx);
            record(entries, max_entries, &cnt, o, 0, cs, 0, 0.f);
            continue;
        }
        float ms = 0.f;
        int iters = 0;
        auto step = [&](int* it) {
            fld_solve_info info{};
            fld_status r = fld_step(ctx, s.E, s.T, rho, kappa_R, kappa_P, c_v, ghost_E, dt, &info);
            *it = info.inner_iters;
            return r;
        };
        fld_status ts = time_steps(step, E, T, s, n, st, reps, &ms, &iters);
        fld_destroy(ctx);
        record(entries, max_entries, &cnt, o, 0, ts, iters, ms);
        if (ts == FLD_EHIP) return FLD_EHIP;
        if (ts == FLD_OK && ms < best_ms) {
            best_ms = ms;
            *best = o;
            overall = FLD_OK;
        }
    }
    if (n_entries) *n_entries = cnt;
    return overall;
}

fld_status fld_batch_tune(int32_t nblocks, const int32_t* nx, const int32_t* ny, const double* dx, const double* dy,
                          const fld_bc* bc, const fld_options* base, const double* E, const double* T,
                          const double* rho, const double* kappa_R, const double* kappa_P, const double* c_v,
                          const double* ghost_E, double dt, int32_t reps, fld_options* best, int32_t* best_threads,
                          fld_tune_entry* entries, int32_t max_entries, int32_t* n_entries, void* stream) {
    if (nblocks < 1 || !nx || !ny || !best || !best_threads || !E || !T || reps < 1) return FLD_EINVAL;
    fld_options b0;
    if (base) b0 = *base;
    else fld_default_options(&b0);
    hipStream_t st = static_cast<hipStream_t>(stream);
    size_t n = 0;
    for (int k = 0; k < nblocks; ++k) n += (size_t)std::max(0, nx[k]) * std::max(0, ny[k]);
    Scratch s;
    if (hipMalloc(&s.E, std::max<size_t>(n, 1) * sizeof(double)) != hipSuccess ||
        hipMalloc(&s.T, std::max<size_t>(n, 1) * sizeof(double)) != hipSuccess)
        return FLD_ENOMEM;
    int32_t cnt = 0;
    float best_ms = INFINITY;
    fld_status overall = FLD_ENOCONV;
    for (int cm : {64, 32, 16}) {
        fld_options o = b0;
        o.mg_coarse_max = cm;
        o.smoother = FLD_SMOOTH_LINE;
        fld_batch* bt = nullptr;
        fld_status cs = fld_batch_create(&bt, nblocks, nx, ny, dx, dy, bc, &o, stream);
        if (cs != FLD_OK) {
            record(entries, max_entries, &cnt, o, 0, cs, 0, 0.f);
            if (cs == FLD_EINVAL) return cs;
            continue;
        }
        std::vector<fld_solve_info> info(nblocks);
        for (int th : {512, 256, 1024}) {
            if (fld_batch_set_threads(bt, th) != FLD_OK) continue;
            float ms = 0.f;
            int iters = 0;
            auto step = [&](int* it) {
                fld_status r = fld_batch_step(bt, s.E, s.T, rho, kappa_R, kappa_P, c_v, ghost_E, dt, info.data());
                int mx = 0;
                for (const auto& i : info) mx = std::max(mx, (int)i.inner_iters);
                *it = mx;
                return r;
            };
            fld_status ts = time_steps(step, E, T, s, n, st, reps, &ms, &iters);
            record(entries, max_entries, &cnt, o, th, ts, iters, ms);
            if (ts == FLD_EHIP) {
                fld_batch_destroy(bt);
                return FLD_EHIP;
            }
            if (ts == FLD_OK && ms < best_ms) {
                best_ms = ms;
                *best = o;
                *best_threads = th;
                overall = FLD_OK;
            }
        }
        fld_batch_destroy(bt);
    }
    if (n_entries) *n_entries = cnt;
    return overall;
}

}  // extern "C"
