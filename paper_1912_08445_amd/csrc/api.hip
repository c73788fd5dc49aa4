// C ABI of the library (declared in include/nlte.h): input validation, device buffers,
// the trace pipeline, one ALI step and the ALI loop.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>

#include "nlte_internal.h"

using namespace nlte;

namespace {

nlte_status fail(nlte_ctx *c, nlte_status code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                         \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(ctx, NLTE_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

template <typename T>
nlte_status dalloc(nlte_ctx *c, T **p, size_t count)
{
    if (*p) {
        // work that *_dev calls enqueued on a caller's stream may still read the old buffer
        (void)hipDeviceSynchronize();
        (void)hipFree(*p);
        *p = nullptr;
    }
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void **)p, sizeof(T) * count);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, NLTE_E_OOM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    return NLTE_OK;
}

template <typename T>
void dfree(T *&p)
{
    if (p) {
        (void)hipDeviceSynchronize();   // as in dalloc: caller-stream work may still read it
        (void)hipFree(p);
    }
    p = nullptr;
}

// Scratch of the allocation-free formal solve (nlte_formal_solve_noalloc_dev): the
// work-queue counter (first kScratchHead bytes) and the line-coefficient staging, in the
// code object's global memory, one copy per device, alive until the process ends.  Host
// code never names the array after set-up: it uses the device address that
// hipGetSymbolAddress returned for that device (scratch_ptr).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchHead = 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_rc[kMaxDevices] = {};
bool g_scratch_done[kMaxDevices] = {};

// Device address of this device's scratch array, looked up once per device with that
// device current; the return code of the lookup is kept for the entry point's error.
void scratch_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_done[device]) return;
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    g_scratch_rc[device] = e;
    g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
    g_scratch_done[device] = true;
}

bool finite_all(const double *a, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

hipStream_t pick(nlte_ctx *c, void *stream) { return stream ? (hipStream_t)stream : c->stream; }

// Time a launch with HIP events on its stream when profiling is on.
template <typename F>
hipError_t timed(nlte_ctx *c, KernelStat &st, hipStream_t s, F &&launch)
{
    if (!c->params.profile) return launch();
    hipError_t e = hipEventRecord(c->ev0, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(c->ev1, s);
    if (e != hipSuccess) return e;
    e = hipEventSynchronize(c->ev1);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, c->ev0, c->ev1);
    st.ms += ms;
    st.launches += 1;
    return e;
}

nlte_status need(nlte_ctx *c, bool traced)
{
    if (!c) return NLTE_E_INVALID_ARG;
    if (!c->have_species) return fail(c, NLTE_E_STATE, "nlte_set_species has not been called");
    if (!c->have_model) return fail(c, NLTE_E_STATE, "nlte_set_models has not been called");
    if (!c->have_rays) return fail(c, NLTE_E_STATE, "nlte_set_rays has not been called");
    if (!c->have_quad) return fail(c, NLTE_E_STATE, "nlte_set_quadrature has not been called");
    if (traced && !c->traced) return fail(c, NLTE_E_STATE, "nlte_trace has not been called");
    return NLTE_OK;
}

// Boundary intensity B_nu(t_cmb) at every line-centre frequency.
nlte_status upload_ibdy(nlte_ctx *c)
{
    if (!c->have_species) return NLTE_OK;
    std::vector<double> ib(c->n_lines);
    for (int l = 0; l < c->n_lines; ++l) {
        double nu = c->nu[l];
        ib[l] = 2.0 * kH * nu * nu * nu / (kC * kC) / expm1(kH * nu / (kKB * c->params.t_cmb));
    }
    nlte_status st = dalloc(c, &c->d_ibdy, c->n_lines);
    if (st) return st;
    HIPCHK(c, hipMemcpy(c->d_ibdy, ib.data(), sizeof(double) * c->n_lines, hipMemcpyHostToDevice));
    return NLTE_OK;
}

// Work buffers sized for the current model and species.
nlte_status ensure_work(nlte_ctx *c)
{
    const int64_t P = c->P;
    const size_t lcbytes = (size_t)P * c->n_lines * sizeof(double2);
    nlte_status st;
    if ((st = dalloc(c, (char **)&c->d_lc, lcbytes))) return st;
    if ((st = dalloc(c, &c->d_pops_a, (size_t)P * c->n_lev))) return st;
    if ((st = dalloc(c, &c->d_pops_b, (size_t)P * c->n_lev))) return st;
    if ((st = dalloc(c, &c->d_J, (size_t)P * c->n_lines))) return st;
    if ((st = dalloc(c, &c->d_Jeff, (size_t)P * c->n_lines))) return st;
    if ((st = dalloc(c, &c->d_L, (size_t)P * c->n_lines))) return st;
    if ((st = dalloc(c, &c->d_flags, (size_t)P))) return st;
    c->n_partials_cap = stateq_blocks(P);
    if ((st = dalloc(c, &c->d_partials, (size_t)c->n_partials_cap))) return st;
    return NLTE_OK;
}

// Register budget (waves per SIMD), far-wing collapse, LDS staging depth and work
// distribution of a formal-solve launch with a.lines_per_wave / a.ngrp lines per lane.
void set_launch_shape(nlte_ctx *c, SolveArgs &a, bool fp32)
{
    const int lpl = a.lines_per_wave / a.ngrp;
    // by rule: 3 waves per SIMD in FP32 and up to two lines per lane in FP64, else 2
    // (measured on the disc: the whole register file for one wave removes the spills of
    // five FP64 lines per lane but leaves too little to hide latency; five FP64 lines at
    // three waves spill inside the node loops; five FP32 lines fit three waves with a few
    // spills outside them, and the third wave takes the disc's FP32 sweep from 4.0 to 3.5 s)
    a.waves = (c->cfg.waves >= 1 && c->cfg.waves <= 3) ? c->cfg.waves : ((lpl <= 2 || fp32) ? 3 : 2);
    // long-segment mode (profile recurrence, far-wing collapse) where sub-step segments are
    // long: more than two elimination steps per cached cell on average
    a.collapse = c->cfg.long_seg >= 0 ? c->cfg.long_seg : (c->total_steps > 2 * c->total_cells ? 1 : 0);
    // the most staged nodes whose LDS keeps the register budget's occupancy (160 KiB per CU):
    // dynamic and static bytes in the units the hardware allocates (counted without them, the
    // disc's FP32 form took 48 nodes and lost one wave per CU to the rounding: 3.40 s per
    // sweep against 3.26 s at 40)
    const size_t budget = (size_t)160 * 1024 / (size_t)(4 * a.waves);
    auto lds = [&](int n) {
        const size_t b = (fp32 ? formal_solve_lds_f32(lpl, n) : formal_solve_lds_f64(lpl, n)) + kFsStaticLds;
        return (b + kLdsGranule - 1) / kLdsGranule * kLdsGranule;
    };
    int ns = kWave;
    while (ns > 16 && lds(ns) > budget) ns -= 8;
    if (c->cfg.ns >= 2 && c->cfg.ns <= kWave) ns = c->cfg.ns;
    a.ns = ns;
    a.persistent = c->cfg.persistent;
    a.tile = (c->cfg.tile >= 1 && c->cfg.tile <= 16) ? c->cfg.tile : 1;
}

SolveArgs solve_args(nlte_ctx *c, double *J, double *Jeff, double *L)
{
    SolveArgs a{};
    a.cell = c->d_cell;
    a.lc = c->d_lc;
    a.roff = c->d_roff;
    a.rcells = c->d_rcells;
    a.dir = c->d_dir;
    a.pair_r = c->d_pair_r;
    a.anti = c->d_anti;
    a.qx = c->d_qx;
    a.qw = c->d_qw;
    a.ibdy = c->d_ibdy;
    a.f_sub = c->params.f_sub;
    a.xq_max = c->xq_max;
    a.norm = 2.0 / (double)c->n_rays;
    a.exec_steps = c->params.profile ? c->d_exec : nullptr;
    a.P = c->P;
    a.n_rays = c->n_rays;
    a.n_pairs = c->n_pairs;
    a.n_q = c->n_q;
    a.n_lines = c->n_lines;
    // A wave takes one or two groups of n_q lanes (one frequency each) and LPL lines per
    // group.  By rule: the fewest waves per point (each wave stages the point's rays and
    // evaluates the profile once per node and frequency for all its lines), then the
    // fewest lines per lane that keep that count (the least register state per lane).
    const int ngrp = (2 * c->n_q <= kWave) ? 2 : 1;
    a.ngrp = ngrp;
    a.fchunks = (c->n_q <= kWave) ? 1 : (c->n_q + kWave - 1) / kWave;
    const int waves_min = (c->n_lines + ngrp * kMaxLpl - 1) / (ngrp * kMaxLpl);
    int lpl = (c->n_lines + ngrp * waves_min - 1) / (ngrp * waves_min);
    // an explicit choice, capped at the lines one lane group can need
    if (c->cfg.lpl >= 1 && c->cfg.lpl <= kMaxLpl) lpl = std::min(c->cfg.lpl, (c->n_lines + ngrp - 1) / ngrp);
    a.lines_per_wave = ngrp * lpl;
    a.groups = (c->n_lines + a.lines_per_wave - 1) / a.lines_per_wave;
    set_launch_shape(c, a, c->params.precision == NLTE_PREC_FP32_BULK);
    a.n_blocks = c->P * a.groups;
    a.J = J;
    a.Jeff = Jeff;
    a.L = L;
    a.model_done = nullptr;
    a.model_of = c->d_model_of;
    a.order = c->d_order;
    a.work_counter = c->d_work_counter;
    return a;
}

// Captured ALI iterations depend on every buffer and parameter; drop them on any change.
void drop_graphs(nlte_ctx *c)
{
    for (int i = 0; i < 2; ++i) {
        if (c->graph_exec[i]) (void)hipGraphExecDestroy(c->graph_exec[i]);
        c->graph_exec[i] = nullptr;
        c->graph_buf[i] = nullptr;
    }
}

// Line coefficients and the formal solve.  ali: skip points of converged models.
// capture: enqueue only (no per-kernel event timing, which would synchronise).
// sc (nullable): caller-provided staging and counter in place of the context's buffers;
// then nothing is timed, counted or allocated.
struct FsScratch {
    void *lc;
    unsigned long long *counter;
};

nlte_status formal_solve_impl(nlte_ctx *c, const double *d_pops, double *d_J, double *d_Jeff,
                              double *d_L, hipStream_t s, bool ali = false, bool capture = false,
                              const FsScratch *sc = nullptr)
{
    const int fp32 = c->params.precision == NLTE_PREC_FP32_BULK;
    void *lcbuf = sc ? sc->lc : c->d_lc;
    int64_t *maser = sc ? nullptr : c->d_maser;
    auto lc = [&] { return launch_line_coef(c->sp, c->d_cell, d_pops, c->P, fp32, lcbuf, maser, s); };
    HIPCHK(c, capture ? lc() : timed(c, c->st_line_coef, s, lc));
    SolveArgs a = solve_args(c, d_J, d_Jeff, d_L);
    if (sc) {
        a.lc = sc->lc;
        a.work_counter = sc->counter;
        a.exec_steps = nullptr;
    }
    if (ali) a.model_done = c->d_model_done;
    if (a.persistent) HIPCHK(c, launch_fill_u64(a.work_counter, 1, 0ull, s));
    auto fs = [&] { return launch_formal_solve(a, c->cfg, fp32, s); };
    HIPCHK(c, capture ? fs() : timed(c, c->st_formal, s, fs));
    return NLTE_OK;
}

nlte_status stateq_impl(nlte_ctx *c, const double *d_old, const double *d_J, const double *d_Jeff,
                        const double *d_L, double *d_new, uint8_t *d_flags, ConvResult *d_conv,
                        hipStream_t s, bool ali = false, bool capture = false)
{
    const int64_t nb = stateq_blocks(c->P);
    auto sq = [&] {
        return launch_stateq(c->sp, c->d_cell, c->d_nh2, c->d_T, c->P, c->params.use_alo, d_old, d_J, d_Jeff,
                             d_L, d_new, d_flags, c->d_partials, nb, ali ? c->d_model_done : nullptr,
                             c->d_model_of, ali ? c->d_model_change : nullptr, s);
    };
    HIPCHK(c, capture ? sq() : timed(c, c->st_stateq, s, sq));
    if (d_conv) HIPCHK(c, launch_conv_final(c->d_partials, nb, d_conv, s));
    return NLTE_OK;
}

// One ALI iteration cur -> nxt with per-model convergence; ends with the number of
// models still iterating and the change summary in pinned host memory.
nlte_status enqueue_iteration(nlte_ctx *c, const double *cur, double *nxt, hipStream_t s, bool capture)
{
    nlte_status st;
    HIPCHK(c, launch_fill_u64(c->d_model_change, c->n_models, 0ull, s));
    HIPCHK(c, launch_fill_u64(reinterpret_cast<unsigned long long *>(c->d_maser), 1, 0ull, s));
    HIPCHK(c, launch_fill_u8(reinterpret_cast<uint8_t *>(c->d_active), sizeof(int32_t), 0, s));
    if ((st = formal_solve_impl(c, cur, c->d_J, c->d_Jeff, c->d_L, s, true, capture))) return st;
    if ((st = stateq_impl(c, cur, c->d_J, c->d_Jeff, c->d_L, nxt, c->d_flags, c->d_conv, s, true, capture)))
        return st;
    HIPCHK(c, launch_model_update(c->n_models, c->d_model_change, c->d_model_done, c->d_model_iters,
                                  c->d_model_last, c->params.tol, c->d_active, s));
    HIPCHK(c, hipMemcpyAsync(c->h_conv, c->d_conv, sizeof(ConvResult), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(c->h_active, c->d_active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    return NLTE_OK;
}

// Capture the iteration cur -> nxt as a graph (once per buffer pair and parameter set).
nlte_status ensure_graph(nlte_ctx *c, int slot, const double *cur, double *nxt)
{
    if (c->graph_exec[slot] && c->graph_buf[slot] == cur) return NLTE_OK;
    if (c->graph_exec[slot]) (void)hipGraphExecDestroy(c->graph_exec[slot]);
    c->graph_exec[slot] = nullptr;
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    nlte_status st = enqueue_iteration(c, cur, nxt, c->stream, true);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(c, NLTE_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph_exec[slot], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, NLTE_E_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    c->graph_buf[slot] = cur;
    return NLTE_OK;
}


// ------------------------------------------------------------------ warm start helpers

// Largest batch of one gradient evaluation: its layer inputs and output gradients take
// 2400 bytes per row (157 MB at the limit).
constexpr int kMlpMaxRows = 1 << 16;

MlpDims mlp_dims(int n_out)
{
    MlpDims d{};
    const int ins[4] = {8, 128, 128, 128};
    const int outs[4] = {128, 128, 128, n_out};
    int64_t off = 0;
    for (int l = 0; l < 4; ++l) {
        d.in[l] = ins[l];
        d.out[l] = outs[l];
        d.w_off[l] = off;
        off += (int64_t)ins[l] * outs[l];
        d.b_off[l] = off;
        off += outs[l];
    }
    d.n_params = off;
    return d;
}

nlte_status need_mlp(nlte_ctx *c)
{
    if (!c) return NLTE_E_INVALID_ARG;
    if (!c->mlp.ready) return fail(c, NLTE_E_STATE, "the warm-start network has no weights (nlte_mlp_init or nlte_mlp_set_weights)");
    return NLTE_OK;
}

// Allocate the network state for n_out outputs and reset the optimiser.
nlte_status mlp_alloc(nlte_ctx *c, int n_out)
{
    if (n_out < 1 || n_out > kMaxLev) return fail(c, NLTE_E_INVALID_ARG, "n_out must be in 1..16");
    MlpState &m = c->mlp;
    m.dims = mlp_dims(n_out);
    const int64_t np = m.dims.n_params;
    nlte_status st;
    if ((st = dalloc(c, &m.d_theta, np))) return st;
    if ((st = dalloc(c, &m.d_m, np))) return st;
    if ((st = dalloc(c, &m.d_v, np))) return st;
    if ((st = dalloc(c, &m.d_grad, np))) return st;
    if ((st = dalloc(c, (char **)&m.d_frags, (size_t)mlp_frag_count() * 64 * 16))) return st;
    if (!m.d_bad && (st = dalloc(c, &m.d_bad, 1))) return st;
    HIPCHK(c, hipMemset(m.d_m, 0, sizeof(float) * np));
    HIPCHK(c, hipMemset(m.d_v, 0, sizeof(float) * np));
    m.batch_cap = 0;
    dfree(m.d_gpart);
    dfree(m.d_lpart);
    dfree(m.d_ht);
    dfree(m.d_dzt);
    m.rows_cap = 0;
    dfree(m.d_x);
    dfree(m.d_y);
    m.step = 0;
    return NLTE_OK;
}

nlte_status mlp_upload(nlte_ctx *c, const std::vector<float> &theta)
{
    MlpState &m = c->mlp;
    HIPCHK(c, hipMemcpy(m.d_theta, theta.data(), sizeof(float) * theta.size(), hipMemcpyHostToDevice));
    HIPCHK(c, launch_mlp_pack(m.d_theta, m.dims, m.d_frags, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    m.ready = true;
    return NLTE_OK;
}

// Training buffers for batches of up to `batch` rows.
nlte_status mlp_ensure_batch(nlte_ctx *c, int batch)
{
    MlpState &m = c->mlp;
    if (batch <= m.batch_cap) return NLTE_OK;
    nlte_status st;
    if ((st = dalloc(c, &m.d_gpart, (size_t)mlp_train_chunks(batch) * m.dims.n_params))) return st;
    if ((st = dalloc(c, &m.d_lpart, (size_t)mlp_train_ld(batch) / 16))) return st;
    if ((st = dalloc(c, &m.d_ht, mlp_train_ht_count(batch)))) return st;
    if ((st = dalloc(c, &m.d_dzt, mlp_train_dzt_count(batch)))) return st;
    m.batch_cap = batch;
    return NLTE_OK;
}

nlte_status mlp_ensure_rows(nlte_ctx *c, int64_t rows)
{
    MlpState &m = c->mlp;
    if (rows <= m.rows_cap) return NLTE_OK;
    nlte_status st;
    if ((st = dalloc(c, &m.d_x, (size_t)rows * 8))) return st;
    if ((st = dalloc(c, &m.d_y, (size_t)rows * 16))) return st;
    m.rows_cap = rows;
    return NLTE_OK;
}

nlte_status mlp_ensure_points(nlte_ctx *c)
{
    MlpState &m = c->mlp;
    if (c->P <= m.pred_cap) return NLTE_OK;
    nlte_status st;
    if ((st = dalloc(c, &m.d_feat, (size_t)c->P * 8))) return st;
    if ((st = dalloc(c, &m.d_xp, (size_t)c->P * 8))) return st;
    if ((st = dalloc(c, &m.d_yp, (size_t)c->P * 16))) return st;
    if ((st = dalloc(c, &m.d_pred, (size_t)c->P * kMaxLev))) return st;
    m.pred_cap = c->P;
    return NLTE_OK;
}

nlte_status features_impl(nlte_ctx *c, double *d_F, hipStream_t s)
{
    HIPCHK(c, timed(c, c->st_features, s, [&] {
        return launch_features(c->d_cell, c->d_nh2, c->d_T, c->d_nbr, c->k, c->d_roff, c->d_rcells, c->d_dir,
                               c->n_rays, c->P, d_F, s);
    }));
    return NLTE_OK;
}

// Features -> standardised inputs -> network (departures from LTE) -> populations, over LTE populations for
// points whose prediction is not finite.  The count of those lands in m.d_bad.
nlte_status predict_impl(nlte_ctx *c, double *d_pops, hipStream_t s)
{
    MlpState &m = c->mlp;
    nlte_status st;
    if ((st = mlp_ensure_points(c))) return st;
    if ((st = features_impl(c, m.d_feat, s))) return st;
    HIPCHK(c, launch_mlp_standardise(m.d_feat, m.norm, c->P, m.d_xp, s));
    HIPCHK(c, timed(c, c->st_mlp_forward, s,
                    [&] { return launch_mlp_forward(m.d_frags, m.d_theta, m.dims, m.d_xp, c->P, m.d_yp, s); }));
    HIPCHK(c, launch_fill_u64(m.d_bad, 1, 0ull, s));
    HIPCHK(c, launch_lte(c->sp, c->d_cell, c->d_T, c->P, d_pops, s));
    HIPCHK(c, launch_mlp_populations(c->sp, m.d_yp, c->d_cell, c->d_T, c->P, d_pops, m.d_bad, s));
    return NLTE_OK;
}

// Optimiser steps on device rows X [n][8], T [n][n_out].
nlte_status train_impl(nlte_ctx *c, const float *d_X, const float *d_T, int64_t n, const nlte_train_params *tp,
                       float *d_loss, hipStream_t s)
{
    MlpState &m = c->mlp;
    nlte_status st;
    if ((st = mlp_ensure_batch(c, tp->batch))) return st;
    const float inv_count = (float)(1.0 / ((double)tp->batch * m.dims.out[3]));
    for (int64_t i = 0; i < tp->steps; ++i) {
        const int64_t t = ++m.step;
        const int64_t start = (int64_t)(((__int128)(t - 1) * tp->batch) % n);
        HIPCHK(c, timed(c, c->st_mlp_train, s, [&] {
            return launch_mlp_train(m.d_frags, m.d_theta, m.dims, d_X, d_T, n, start, tp->batch, m.d_ht,
                                    m.d_dzt, m.d_gpart, m.d_lpart, s);
        }));
        const float c1 = (float)(1.0 / (1.0 - pow(tp->beta1, (double)t)));
        const float c2 = (float)(1.0 / (1.0 - pow(tp->beta2, (double)t)));
        HIPCHK(c, timed(c, c->st_mlp_update, s, [&] {
            return launch_mlp_update(m.d_theta, m.d_m, m.d_v, m.d_frags, m.dims, m.d_gpart, tp->batch, 1,
                                     (float)tp->lr, (float)tp->beta1, (float)tp->beta2, (float)tp->eps, c1, c2,
                                     m.d_lpart, inv_count, d_loss ? d_loss + i : nullptr, nullptr, s);
        }));
    }
    return NLTE_OK;
}

nlte_status check_train_params(nlte_ctx *c, int64_t n, const nlte_train_params *tp)
{
    if (!tp || n < 1 || tp->steps < 0 || tp->batch < 1 || tp->batch > kMlpMaxRows || !(tp->lr >= 0.0) ||
        !(tp->beta1 >= 0.0 && tp->beta1 < 1.0) || !(tp->beta2 >= 0.0 && tp->beta2 < 1.0) || !(tp->eps >= 0.0))
        return fail(c, NLTE_E_INVALID_ARG, "invalid training parameters (n >= 1, batch 1..65536, 0 <= beta < 1, lr, eps >= 0)");
    return NLTE_OK;
}

// SplitMix64 (Steele, Lea and Flood 2014): the state advances by the golden-ratio
// increment and each output is the state passed through two xor-shift-multiply rounds.
uint64_t splitmix64(uint64_t &state)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}


// Ng work arrays for the current model(s) and ng_every.
nlte_status ensure_ng(nlte_ctx *c)
{
    const int M = c->params.ng_every;
    const int64_t need = (int64_t)M * c->P * c->n_lev;
    nlte_status st;
    if (need > c->ng_hist_elems) {
        if ((st = dalloc(c, &c->d_ng_hist, (size_t)need))) return st;
        c->ng_hist_elems = need;
    }
    if (c->n_models > c->ng_models_cap || !c->d_ng_rej) {
        const int K = kNgMaxM - 2;
        if ((st = dalloc(c, &c->d_ng_part, (size_t)c->n_models * ng_chunks() * (K * (K + 1) / 2 + K)))) return st;
        if ((st = dalloc(c, &c->d_ng_coef, (size_t)c->n_models * (kNgMaxM - 1)))) return st;
        if ((st = dalloc(c, &c->d_ng_ok, (size_t)c->n_models))) return st;
        if ((st = dalloc(c, &c->d_ng_rej, 1))) return st;
        c->ng_models_cap = c->n_models;
    }
    return NLTE_OK;
}

// ------------------------------------------------------------------ band ALO helpers

// Buffers of the band formal solve and the coupled solve for the current model, rays
// and species, and the first cells of the walks.
nlte_status ensure_band(nlte_ctx *c)
{
    const int64_t P = c->P;
    const int n = c->n_lev, nl = c->n_lines, R = c->n_rays;
    const int64_t dims[5] = {P, n, nl, R, c->n_models};
    nlte_status st;
    if (memcmp(dims, c->band_dims, sizeof dims) != 0) {
        if ((st = dalloc(c, &c->d_first, (size_t)P * R))) return st;
        if ((st = dalloc(c, &c->d_Jb, (size_t)P * nl))) return st;
        if ((st = dalloc(c, &c->d_Ld, (size_t)P * nl))) return st;
        if ((st = dalloc(c, &c->d_Ln, (size_t)P * nl * R))) return st;
        if ((st = dalloc(c, &c->d_bLU, (size_t)P * n * n))) return st;
        if ((st = dalloc(c, &c->d_bcpl, (size_t)P * nl * R))) return st;
        if ((st = dalloc(c, &c->d_bx0, (size_t)P * n))) return st;
        if ((st = dalloc(c, &c->d_bpiv, (size_t)P * n))) return st;
        if ((st = dalloc(c, &c->d_bvec, (size_t)P * n * 8))) return st;
        if ((st = dalloc(c, &c->d_bpart, (size_t)band_dot_blocks(P) * 3))) return st;
        if ((st = dalloc(c, &c->d_bdot, 3))) return st;
        if ((st = dalloc(c, &c->d_bbad, 1))) return st;
        if ((st = dalloc(c, &c->d_bmodel_bad, (size_t)c->n_models))) return st;
        c->h_bmodel_bad.assign((size_t)c->n_models, 0);
        if (!c->h_bdot) HIPCHK(c, hipHostMalloc((void **)&c->h_bdot, sizeof(double) * 3, hipHostMallocDefault));
        if (!c->h_bbad)
            HIPCHK(c, hipHostMalloc((void **)&c->h_bbad, sizeof(unsigned long long), hipHostMallocDefault));
        memcpy(c->band_dims, dims, sizeof dims);
        c->first_valid = false;
    }
    if (!c->first_valid) {
        HIPCHK(c, launch_first_cells(c->d_roff, c->d_rcells, P * R, c->d_first, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->first_valid = true;
    }
    return NLTE_OK;
}

// Band formal solve (FP64 whatever the precision setting): J, Jeff, L as the local one plus
// Jb, Ld, Ln into the context's band buffers.
nlte_status formal_solve_band_impl(nlte_ctx *c, const double *d_pops, double *d_J, double *d_Jeff, double *d_L,
                                   hipStream_t s, bool ali)
{
    HIPCHK(c, launch_line_coef(c->sp, c->d_cell, d_pops, c->P, 0, c->d_lc, c->d_maser, s));
    SolveArgs a = solve_args(c, d_J, d_Jeff, d_L);
    if (a.lines_per_wave / a.ngrp > 2) {   // the band kernel takes one or two lines per lane
        a.lines_per_wave = a.ngrp * 2;
        a.groups = (c->n_lines + a.lines_per_wave - 1) / a.lines_per_wave;
        a.n_blocks = c->P * a.groups;
    }
    {   // its own launch: FP64, a budget of two waves per SIMD, the same segment mode
        const SolveConfig keep = c->cfg;
        c->cfg.waves = 2;
        set_launch_shape(c, a, false);
        c->cfg = keep;
        a.persistent = 0;
        a.tile = 1;
    }
    if (ali) a.model_done = c->d_model_done;
    a.Jb = c->d_Jb;
    a.Ld = c->d_Ld;
    a.Ln = c->d_Ln;
    HIPCHK(c, timed(c, c->st_formal, s, [&] { return launch_formal_solve_band(a, s); }));
    return NLTE_OK;
}

// Weighted inner products (a_k, b_k), k < nd, into c->h_bdot (synchronises s).
nlte_status band_dots(nlte_ctx *c, int nd, const double *a0, const double *b0, const double *a1, const double *b1,
                      const double *a2, const double *b2, hipStream_t s)
{
    DotArgs d{};
    d.a[0] = a0;
    d.b[0] = b0;
    d.a[1] = a1 ? a1 : a0;
    d.b[1] = b1 ? b1 : b0;
    d.a[2] = a2 ? a2 : a0;
    d.b[2] = b2 ? b2 : b0;
    d.nd = nd;
    HIPCHK(c, launch_band_dots(d, c->d_cell, c->n_lev, c->P, c->d_bpart, c->d_bdot, s));
    HIPCHK(c, hipMemcpyAsync(c->h_bdot, c->d_bdot, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return NLTE_OK;
}

// Coupled statistical equilibrium of the band ALO by preconditioned BiCGSTAB (see
// band.hip).  The band is dropped per model (Sec. 6.1): a model with a singular local
// matrix, or whose coupled solution has a population that is not positive and finite,
// takes the local solve (diagonal ALO) and the other models keep the band's populations;
// if the coupled solve itself breaks down or does not converge, every model takes the
// local solve.  Leaves the change partials for launch_conv_final.  *used: models whose
// populations came from the band; *iters: solver steps.
nlte_status stateq_band_impl(nlte_ctx *c, const double *d_old, const double *d_J, const double *d_Jeff,
                             const double *d_L, double *d_new, uint8_t *d_flags, hipStream_t s, bool ali, int *used,
                             int *iters)
{
    const int n = c->n_lev;
    const int64_t N = c->P * n;
    const double tol = 1e-13;
    *used = 0;
    *iters = 0;
    BandArgs b{};
    b.Jb = c->d_Jb;
    b.Ld = c->d_Ld;
    b.Ln = c->d_Ln;
    b.first = c->d_first;
    b.done = ali ? c->d_model_done : nullptr;
    b.model_of = c->d_model_of;
    b.LU = c->d_bLU;
    b.piv = c->d_bpiv;
    b.cpl = c->d_bcpl;
    b.x0 = c->d_bx0;
    b.bad = c->d_bbad;
    b.model_bad = c->d_bmodel_bad;
    b.P = c->P;
    b.R = c->n_rays;
    double *x = c->d_bvec, *r = x + N, *r0 = r + N, *p = r0 + N, *v = p + N, *sv = v + N, *t = sv + N, *w = t + N;
    HIPCHK(c, launch_fill_u64(c->d_bbad, 1, 0ull, s));
    HIPCHK(c, launch_fill_u8(c->d_bmodel_bad, c->n_models, 0, s));
    HIPCHK(c, launch_band_setup(b, c->sp, c->d_cell, c->d_nh2, c->d_T, d_old, s));
    HIPCHK(c, launch_band_mask(b, c->n_lines, s));
    nlte_status st;
    // x = K^-1 b; r = K^-1 b - (I + K^-1 C) x = -(K^-1 C) x
    HIPCHK(c, launch_band_lin(x, 1.0, c->d_bx0, 0.0, c->d_bx0, 0.0, nullptr, N, s));
    HIPCHK(c, launch_band_apply(b, c->sp, x, w, s));
    HIPCHK(c, launch_band_lin(r, 1.0, x, -1.0, w, 0.0, nullptr, N, s));
    HIPCHK(c, launch_band_lin(r0, 1.0, r, 0.0, r, 0.0, nullptr, N, s));
    HIPCHK(c, launch_band_lin(p, 0.0, r, 0.0, r, 0.0, nullptr, N, s));
    HIPCHK(c, launch_band_lin(v, 0.0, r, 0.0, r, 0.0, nullptr, N, s));
    if ((st = band_dots(c, 3, r0, r, r, r, x, x, s))) return st;
    double rho = 1.0, alpha = 1.0, omega = 1.0, rho1 = c->h_bdot[0];
    bool ok = true;
    bool conv = !(c->h_bdot[2] > 0.0) || c->h_bdot[1] <= tol * tol * c->h_bdot[2];
    for (int it = 0; it < 200 && !conv && ok; ++it) {
        *iters = it + 1;
        if (!(rho1 != 0.0) || !std::isfinite(rho1)) {
            ok = false;
            break;
        }
        const double beta = (rho1 / rho) * (alpha / omega);
        HIPCHK(c, launch_band_lin(p, 1.0, r, beta, p, -beta * omega, v, N, s));
        HIPCHK(c, launch_band_apply(b, c->sp, p, v, s));
        if ((st = band_dots(c, 1, r0, v, nullptr, nullptr, nullptr, nullptr, s))) return st;
        const double sigma = c->h_bdot[0];
        if (!(sigma != 0.0) || !std::isfinite(sigma)) {
            ok = false;
            break;
        }
        alpha = rho1 / sigma;
        HIPCHK(c, launch_band_lin(sv, 1.0, r, -alpha, v, 0.0, nullptr, N, s));
        if ((st = band_dots(c, 2, sv, sv, x, x, nullptr, nullptr, s))) return st;
        if (c->h_bdot[0] <= tol * tol * c->h_bdot[1]) {
            HIPCHK(c, launch_band_lin(x, 1.0, x, alpha, p, 0.0, nullptr, N, s));
            conv = true;
            break;
        }
        HIPCHK(c, launch_band_apply(b, c->sp, sv, t, s));
        if ((st = band_dots(c, 2, t, sv, t, t, nullptr, nullptr, s))) return st;
        if (!(c->h_bdot[1] > 0.0)) {
            ok = false;
            break;
        }
        omega = c->h_bdot[0] / c->h_bdot[1];
        HIPCHK(c, launch_band_lin(x, 1.0, x, alpha, p, omega, sv, N, s));
        HIPCHK(c, launch_band_lin(r, 1.0, sv, -omega, t, 0.0, nullptr, N, s));
        if ((st = band_dots(c, 3, r0, r, r, r, x, x, s))) return st;
        rho = rho1;
        rho1 = c->h_bdot[0];
        conv = c->h_bdot[1] <= tol * tol * c->h_bdot[2];
        if (!(omega != 0.0)) ok = false;
    }
    ok = ok && conv;
    int n_bad = c->n_models;
    if (ok) {
        HIPCHK(c, launch_band_check_models(x, n, c->P, c->d_model_of, c->d_bmodel_bad, s));
        HIPCHK(c, hipMemcpyAsync(c->h_bmodel_bad.data(), c->d_bmodel_bad, (size_t)c->n_models, hipMemcpyDeviceToHost,
                                 s));
        HIPCHK(c, hipStreamSynchronize(s));
        n_bad = 0;
        for (uint8_t f : c->h_bmodel_bad) n_bad += f != 0;
    }
    auto local = [&](double *out, ConvPartial *parts, unsigned long long *change) {
        return launch_stateq(c->sp, c->d_cell, c->d_nh2, c->d_T, c->P, c->params.use_alo, d_old, d_J, d_Jeff, d_L,
                             out, d_flags, parts, stateq_blocks(c->P), ali ? c->d_model_done : nullptr,
                             c->d_model_of, change, s);
    };
    if (n_bad == c->n_models) {
        // the band gave no model physical populations: the local solve everywhere
        HIPCHK(c, local(d_new, c->d_partials, ali ? c->d_model_change : nullptr));
        return NLTE_OK;
    }
    if (n_bad > 0) HIPCHK(c, local(r0, nullptr, nullptr));   // r0 is free once the solve is done
    *used = c->n_models - n_bad;
    HIPCHK(c, launch_band_finish(x, n_bad > 0 ? r0 : nullptr, n_bad > 0 ? c->d_bmodel_bad : nullptr, d_old, c->d_cell, n,
                                 c->P, d_new, d_flags, c->d_partials, ali ? c->d_model_done : nullptr, c->d_model_of,
                                 ali ? c->d_model_change : nullptr, s));
    return NLTE_OK;
}

// One band-ALO iteration cur -> nxt (not captured: the solver reads scalars back).
nlte_status iteration_band(nlte_ctx *c, const double *cur, double *nxt, hipStream_t s, int *used)
{
    nlte_status st;
    int iters = 0;
    HIPCHK(c, launch_fill_u64(c->d_model_change, c->n_models, 0ull, s));
    HIPCHK(c, launch_fill_u64(reinterpret_cast<unsigned long long *>(c->d_maser), 1, 0ull, s));
    HIPCHK(c, launch_fill_u8(reinterpret_cast<uint8_t *>(c->d_active), sizeof(int32_t), 0, s));
    if ((st = formal_solve_band_impl(c, cur, c->d_J, c->d_Jeff, c->d_L, s, true))) return st;
    if ((st = stateq_band_impl(c, cur, c->d_J, c->d_Jeff, c->d_L, nxt, c->d_flags, s, true, used, &iters))) return st;
    HIPCHK(c, launch_conv_final(c->d_partials, stateq_blocks(c->P), c->d_conv, s));
    HIPCHK(c, launch_model_update(c->n_models, c->d_model_change, c->d_model_done, c->d_model_iters,
                                  c->d_model_last, c->params.tol, c->d_active, s));
    HIPCHK(c, hipMemcpyAsync(c->h_conv, c->d_conv, sizeof(ConvResult), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(c->h_active, c->d_active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    return NLTE_OK;
}

// ------------------------------------------------------------------ scattering helpers

nlte_status need_scat(nlte_ctx *c)
{
    if (!c->scat_on) return fail(c, NLTE_E_STATE, "nlte_set_scattering has not been called");
    if (!c->q_ascending)
        return fail(c, NLTE_E_INVALID_ARG, "the scattering solve needs an ascending quadrature");
    return NLTE_OK;
}

// Formal solve with scattering (FP64 whatever the precision setting): J, Jeff, L and the new
// J_nu from the previous one.
nlte_status formal_solve_scat_impl(nlte_ctx *c, const double *d_pops, const double *d_jin, double *d_J,
                                   double *d_Jeff, double *d_L, double *d_jout, hipStream_t s, bool ali)
{
    HIPCHK(c, launch_line_coef(c->sp, c->d_cell, d_pops, c->P, 0, c->d_lc, c->d_maser, s));
    ScatArgs a{};
    a.cell = c->d_cell;
    a.lc = c->d_lc;
    a.roff = c->d_roff;
    a.rcells = c->d_rcells;
    a.dir = c->d_dir;
    a.pair_r = c->d_pair_r;
    a.anti = c->d_anti;
    a.qx = c->d_qx;
    a.qw = c->d_qw;
    a.ibdy = c->d_ibdy;
    a.chi_sca = c->d_chi_sca;
    a.chi_dip = c->dip_on ? c->d_chi_dip : nullptr;
    a.Jin = d_jin;
    a.Jout = d_jout;
    a.J = d_J;
    a.Jeff = d_Jeff;
    a.L = d_L;
    a.f_sub = c->params.f_sub;
    a.norm = 2.0 / (double)c->n_rays;
    a.inv_rays = 1.0 / (double)c->n_rays;
    a.P = c->P;
    a.n_rays = c->n_rays;
    a.n_pairs = c->n_pairs;
    a.n_q = c->n_q;
    a.n_lines = c->n_lines;
    a.q_uniform = c->q_uniform ? 1 : 0;
    a.q_inv_h = c->q_inv_h;
    if (ali) {
        a.model_done = c->d_model_done;
        a.model_of = c->d_model_of;
    }
    HIPCHK(c, timed(c, c->st_formal, s, [&] { return launch_formal_solve_scat(a, s); }));
    return NLTE_OK;
}

nlte_status ensure_jnu(nlte_ctx *c)
{
    const int64_t n = c->P * c->n_lines * c->n_q;
    if (n != c->jnu_elems || !c->d_jnu[0]) {
        nlte_status st;
        if ((st = dalloc(c, &c->d_jnu[0], (size_t)n)) || (st = dalloc(c, &c->d_jnu[1], (size_t)n))) return st;
        c->jnu_elems = n;
    }
    return NLTE_OK;
}

// One ALI iteration with scattering, cur -> nxt (launched eagerly: the J_nu buffers
// alternate).
nlte_status iteration_scat(nlte_ctx *c, const double *cur, double *nxt, hipStream_t s)
{
    nlte_status st;
    const int jin = c->jnu_last;
    HIPCHK(c, launch_fill_u64(c->d_model_change, c->n_models, 0ull, s));
    HIPCHK(c, launch_fill_u64(reinterpret_cast<unsigned long long *>(c->d_maser), 1, 0ull, s));
    HIPCHK(c, launch_fill_u8(reinterpret_cast<uint8_t *>(c->d_active), sizeof(int32_t), 0, s));
    if ((st = formal_solve_scat_impl(c, cur, c->d_jnu[jin], c->d_J, c->d_Jeff, c->d_L, c->d_jnu[jin ^ 1], s, true)))
        return st;
    c->jnu_last = jin ^ 1;
    if ((st = stateq_impl(c, cur, c->d_J, c->d_Jeff, c->d_L, nxt, c->d_flags, c->d_conv, s, true, false))) return st;
    HIPCHK(c, launch_model_update(c->n_models, c->d_model_change, c->d_model_done, c->d_model_iters,
                                  c->d_model_last, c->params.tol, c->d_active, s));
    HIPCHK(c, hipMemcpyAsync(c->h_conv, c->d_conv, sizeof(ConvResult), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(c->h_active, c->d_active, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    return NLTE_OK;
}

}  // namespace

extern "C" {

void nlte_default_params(nlte_params *p)
{
    if (!p) return;
    p->t_cmb = 2.725;
    p->f_sub = 0.25;
    p->tol = 1e-4;
    p->max_iter = 50;
    p->use_alo = 1;
    p->precision = NLTE_PREC_FP64;
    p->profile = 0;
    p->use_graph = 1;
    p->lines_per_lane = 0;
    p->waves_per_simd = 0;
    p->long_segments = -1;
    p->stage_nodes = 0;
    p->tile_points = 0;
    p->persistent = 1;   // measured no slower on every workload (the disc: 4.87 -> 4.65 s)
    p->ng_every = 0;
    p->alo_band = 0;
}

nlte_status nlte_create(nlte_ctx **out, int hip_device)
{
    if (!out) return NLTE_E_INVALID_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return NLTE_E_HIP;
    nlte_ctx *c = new (std::nothrow) nlte_ctx();
    if (!c) return NLTE_E_OOM;
    c->device = hip_device;
    nlte_default_params(&c->params);
    if (hipSetDevice(hip_device) != hipSuccess ||
        // blocking: ordered with the null stream, which callers (torch's default stream) use
        hipStreamCreateWithFlags(&c->stream, hipStreamDefault) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
        hipMalloc((void **)&c->d_maser, sizeof(int64_t)) != hipSuccess ||
        hipMalloc((void **)&c->d_conv, sizeof(ConvResult) * 1025) != hipSuccess ||
        hipHostMalloc((void **)&c->h_conv, sizeof(ConvResult) * 1025, 0) != hipSuccess ||
        hipMalloc((void **)&c->d_active, sizeof(int32_t)) != hipSuccess ||
        hipHostMalloc((void **)&c->h_active, sizeof(int32_t), 0) != hipSuccess ||
        hipMalloc((void **)&c->d_work_counter, sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void **)&c->d_exec, sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(c->d_exec, 0, sizeof(unsigned long long)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        nlte_destroy(c);
        return NLTE_E_HIP;
    }
    scratch_setup(hip_device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) {
        c->n_cu = prop.multiProcessorCount;
        c->device_name = prop.gcnArchName;
    }
    if (c->n_cu <= 0) c->n_cu = 256;
    c->cfg.n_wg = c->n_cu * 16;
    *out = c;
    return NLTE_OK;
}

void nlte_destroy(nlte_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    // *_dev calls enqueue work on the caller's streams that reads the context's buffers
    (void)hipDeviceSynchronize();
    dfree(c->d_exec);
    dfree(c->d_species_mem);
    dfree(c->d_cell);
    dfree(c->d_nh2);
    dfree(c->d_T);
    dfree(c->d_nbr);
    dfree(c->d_bnd);
    dfree(c->d_dir);
    dfree(c->d_pair_r);
    dfree(c->d_anti);
    dfree(c->d_qx);
    dfree(c->d_qw);
    dfree(c->d_ibdy);
    dfree(c->d_roff);
    dfree(c->d_rcells);
    dfree(c->d_lc);
    dfree(c->d_pops_a);
    dfree(c->d_pops_b);
    dfree(c->d_J);
    dfree(c->d_Jeff);
    dfree(c->d_L);
    dfree(c->d_flags);
    dfree(c->d_partials);
    dfree(c->d_conv);
    dfree(c->d_maser);
    dfree(c->d_active);
    dfree(c->d_work_counter);
    dfree(c->d_order);
    dfree(c->d_cost);
    dfree(c->d_model_of);
    dfree(c->d_model_off);
    dfree(c->d_morton);
    dfree(c->d_vch);
    dfree(c->d_chi_sca);
    dfree(c->d_chi_dip);
    dfree(c->d_jnu[0]);
    dfree(c->d_jnu[1]);
    dfree(c->d_first);
    dfree(c->d_Jb);
    dfree(c->d_Ld);
    dfree(c->d_Ln);
    dfree(c->d_bLU);
    dfree(c->d_bcpl);
    dfree(c->d_bx0);
    dfree(c->d_bpiv);
    dfree(c->d_bvec);
    dfree(c->d_bpart);
    dfree(c->d_bdot);
    dfree(c->d_bbad);
    dfree(c->d_bmodel_bad);
    if (c->h_bdot) (void)hipHostFree(c->h_bdot);
    if (c->h_bbad) (void)hipHostFree(c->h_bbad);
    dfree(c->d_ng_hist);
    dfree(c->d_ng_part);
    dfree(c->d_ng_coef);
    dfree(c->d_ng_ok);
    dfree(c->d_ng_rej);
    dfree(c->d_model_done);
    dfree(c->d_model_change);
    dfree(c->d_model_iters);
    dfree(c->d_model_last);
    {
        MlpState &m = c->mlp;
        dfree(m.d_theta);
        dfree(m.d_m);
        dfree(m.d_v);
        dfree(m.d_frags);
        dfree(m.d_gpart);
        dfree(m.d_lpart);
        dfree(m.d_ht);
        dfree(m.d_dzt);
        dfree(m.d_loss);
        dfree(m.d_grad);
        dfree(m.d_x);
        dfree(m.d_y);
        dfree(m.d_feat);
        dfree(m.d_xp);
        dfree(m.d_yp);
        dfree(m.d_pred);
        dfree(m.d_bad);
    }
    drop_graphs(c);
    if (c->h_conv) (void)hipHostFree(c->h_conv);
    if (c->h_active) (void)hipHostFree(c->h_active);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *nlte_last_error(const nlte_ctx *c) { return c ? c->err.c_str() : "null context"; }

nlte_status nlte_set_species(nlte_ctx *c, int n_lev, const double *E, const double *g, double mass,
                             int n_lines, const int32_t *up, const int32_t *lo, const double *A_ul,
                             int n_coll, const int32_t *c_up, const int32_t *c_lo, int n_T,
                             const double *T_K, const double *K_ul)
{
    if (!c) return NLTE_E_INVALID_ARG;
    (void)hipSetDevice(c->device);
    if (n_lev < 2 || n_lev > kMaxLev) return fail(c, NLTE_E_INVALID_ARG, "n_lev out of [2, 16]");
    if (n_lines < 1 || n_lines > kMaxLines) return fail(c, NLTE_E_INVALID_ARG, "n_lines out of [1, 32]");
    if (n_coll < 0 || n_coll > 256) return fail(c, NLTE_E_INVALID_ARG, "n_coll out of [0, 256]");
    if (n_T < 1 || n_T > 256) return fail(c, NLTE_E_INVALID_ARG, "n_T out of [1, 256]");
    if (!E || !g || !up || !lo || !A_ul || !T_K || (n_coll > 0 && (!c_up || !c_lo || !K_ul)))
        return fail(c, NLTE_E_INVALID_ARG, "null species array");
    if (!(mass > 0.0) || !std::isfinite(mass)) return fail(c, NLTE_E_INVALID_ARG, "mass must be > 0");
    if (!finite_all(E, n_lev) || !finite_all(g, n_lev) || !finite_all(A_ul, n_lines) ||
        !finite_all(T_K, n_T) || !finite_all(K_ul, (int64_t)n_coll * n_T))
        return fail(c, NLTE_E_INVALID_ARG, "non-finite species data");
    for (int i = 0; i < n_lev; ++i)
        if (!(g[i] > 0.0)) return fail(c, NLTE_E_INVALID_ARG, "statistical weights must be > 0");
    for (int l = 0; l < n_lines; ++l) {
        if (up[l] < 0 || up[l] >= n_lev || lo[l] < 0 || lo[l] >= n_lev || !(E[up[l]] > E[lo[l]]))
            return fail(c, NLTE_E_INVALID_ARG, "line levels out of range or E_up <= E_lo");
        if (!(A_ul[l] >= 0.0)) return fail(c, NLTE_E_INVALID_ARG, "negative Einstein A");
    }
    for (int i = 0; i < n_coll; ++i)
        if (c_up[i] < 0 || c_up[i] >= n_lev || c_lo[i] < 0 || c_lo[i] >= n_lev || c_up[i] == c_lo[i])
            return fail(c, NLTE_E_INVALID_ARG, "collision levels out of range");
    for (int t = 0; t + 1 < n_T; ++t)
        if (!(T_K[t + 1] > T_K[t])) return fail(c, NLTE_E_INVALID_ARG, "T table not increasing");

    // packed device layout: ints first, then doubles
    const int ni = 2 * n_lines + 2 * n_coll;
    const int nd = 5 * n_lines + 2 * n_lev + n_T + n_coll * n_T;
    std::vector<int32_t> hi(ni);
    std::vector<double> hd(nd);
    c->nu.assign(n_lines, 0.0);
    for (int l = 0; l < n_lines; ++l) {
        hi[l] = up[l];
        hi[n_lines + l] = lo[l];
        double nu = (E[up[l]] - E[lo[l]]) / kH;
        c->nu[l] = nu;
        double Bul = A_ul[l] * kC * kC / (2.0 * kH * nu * nu * nu);
        hd[l] = A_ul[l];
        hd[n_lines + l] = nu;
        hd[2 * n_lines + l] = Bul;
        hd[3 * n_lines + l] = (g[up[l]] / g[lo[l]]) * Bul;
        hd[4 * n_lines + l] = kH * nu / (4.0 * kPi);
    }
    for (int i = 0; i < n_coll; ++i) {
        hi[2 * n_lines + i] = c_up[i];
        hi[2 * n_lines + n_coll + i] = c_lo[i];
    }
    double *dd = hd.data() + 5 * n_lines;
    memcpy(dd, E, sizeof(double) * n_lev);
    memcpy(dd + n_lev, g, sizeof(double) * n_lev);
    memcpy(dd + 2 * n_lev, T_K, sizeof(double) * n_T);
    if (n_coll) memcpy(dd + 2 * n_lev + n_T, K_ul, sizeof(double) * n_coll * n_T);
    const size_t ibytes = ((sizeof(int32_t) * ni + 255) / 256) * 256;
    char *mem = nullptr;
    nlte_status st = dalloc(c, &mem, ibytes + sizeof(double) * nd);
    if (st) return st;
    dfree(c->d_species_mem);
    c->d_species_mem = mem;
    HIPCHK(c, hipMemcpy(mem, hi.data(), sizeof(int32_t) * ni, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(mem + ibytes, hd.data(), sizeof(double) * nd, hipMemcpyHostToDevice));
    const int32_t *di = (const int32_t *)mem;
    const double *ddv = (const double *)(mem + ibytes);
    SpeciesDev &sp = c->sp;
    sp.n_lev = n_lev;
    sp.n_lines = n_lines;
    sp.n_coll = n_coll;
    sp.n_T = n_T;
    sp.mass = mass;
    sp.lu = di;
    sp.ll = di + n_lines;
    sp.cu = di + 2 * n_lines;
    sp.cl = di + 2 * n_lines + n_coll;
    sp.A = ddv;
    sp.nu = ddv + n_lines;
    sp.Bul = ddv + 2 * n_lines;
    sp.Blu = ddv + 3 * n_lines;
    sp.pre = ddv + 4 * n_lines;
    sp.E = ddv + 5 * n_lines;
    sp.g = sp.E + n_lev;
    sp.Ttab = sp.g + n_lev;
    sp.Ktab = sp.Ttab + n_T;
    c->n_lev = n_lev;
    c->n_lines = n_lines;
    c->n_coll = n_coll;
    c->n_T = n_T;
    c->mass = mass;
    drop_graphs(c);
    c->have_species = true;
    c->scat_on = false;     // scattering opacities are per line
    c->dip_on = false;
    c->jnu_last = -1;
    // line widths and work buffers depend on the species: the model must be set again
    c->have_model = false;
    c->traced = false;
    return upload_ibdy(c);
}

nlte_status nlte_set_models(nlte_ctx *c, int n_models, const int64_t *offsets, const double *pos,
                            const double *vel, const double *n_h2, const double *T,
                            const double *v_turb, const double *abundance, int k,
                            const int32_t *nbr, const uint8_t *boundary)
{
    if (!c) return NLTE_E_INVALID_ARG;
    (void)hipSetDevice(c->device);
    if (!c->have_species) return fail(c, NLTE_E_STATE, "call nlte_set_species first");
    if (n_models < 1) return fail(c, NLTE_E_INVALID_ARG, "n_models must be >= 1");
    if (!pos || !vel || !n_h2 || !T || !v_turb || !abundance || !nbr)
        return fail(c, NLTE_E_INVALID_ARG, "null model array");
    if (k < 1 || k > 64) return fail(c, NLTE_E_INVALID_ARG, "k out of [1, 64]");
    if (!offsets) return fail(c, NLTE_E_INVALID_ARG, "offsets required ({0, P} for one model)");
    std::vector<int64_t> off(offsets, offsets + n_models + 1);
    if (off[0] != 0) return fail(c, NLTE_E_INVALID_ARG, "offsets[0] must be 0");
    for (int m = 0; m < n_models; ++m)
        if (off[m + 1] <= off[m]) return fail(c, NLTE_E_INVALID_ARG, "empty or decreasing model");
    const int64_t P = off[n_models];
    if (P < 1 || P > ((int64_t)1 << 31) - 1) return fail(c, NLTE_E_INVALID_ARG, "point count out of range");
    if (!finite_all(pos, 3 * P) || !finite_all(vel, 3 * P) || !finite_all(n_h2, P) ||
        !finite_all(T, P) || !finite_all(v_turb, P) || !finite_all(abundance, P))
        return fail(c, NLTE_E_INVALID_ARG, "non-finite model data");
    for (int64_t p = 0; p < P; ++p)
        if (!(T[p] > 0.0) || n_h2[p] < 0.0 || abundance[p] < 0.0 || v_turb[p] < 0.0)
            return fail(c, NLTE_E_INVALID_ARG, "T must be > 0 and densities, abundances, v_turb >= 0");
    std::vector<int32_t> g(P * (size_t)k);
    for (int m = 0; m < n_models; ++m) {
        const int64_t o = off[m], n = off[m + 1] - off[m];
        for (int64_t p = o; p < o + n; ++p)
            for (int s = 0; s < k; ++s) {
                int32_t v = nbr[p * k + s];
                if (v == -1) {
                    g[p * k + s] = -1;
                    continue;
                }
                if (v < 0 || v >= n) return fail(c, NLTE_E_INVALID_ARG, "neighbour index out of range");
                if (o + v == p) return fail(c, NLTE_E_INVALID_ARG, "point lists itself as neighbour");
                g[p * k + s] = (int32_t)(o + v);
            }
    }
    // device copies
    double *d_pos = nullptr, *d_vel = nullptr, *d_vt = nullptr, *d_X = nullptr;
    nlte_status st;
    if ((st = dalloc(c, &c->d_cell, P)) || (st = dalloc(c, &c->d_nh2, P)) || (st = dalloc(c, &c->d_T, P)) ||
        (st = dalloc(c, &c->d_nbr, P * (size_t)k)) || (st = dalloc(c, &d_pos, 3 * P)) ||
        (st = dalloc(c, &d_vel, 3 * P)) || (st = dalloc(c, &d_vt, P)) || (st = dalloc(c, &d_X, P))) {
        dfree(d_pos);
        dfree(d_vel);
        dfree(d_vt);
        dfree(d_X);
        return st;
    }
    dfree(c->d_bnd);
    hipError_t e = hipSuccess;
    auto cp = [&](void *d, const void *h, size_t b) {
        if (e == hipSuccess) e = hipMemcpy(d, h, b, hipMemcpyHostToDevice);
    };
    cp(d_pos, pos, sizeof(double) * 3 * P);
    cp(d_vel, vel, sizeof(double) * 3 * P);
    cp(c->d_nh2, n_h2, sizeof(double) * P);
    cp(c->d_T, T, sizeof(double) * P);
    cp(d_vt, v_turb, sizeof(double) * P);
    cp(d_X, abundance, sizeof(double) * P);
    cp(c->d_nbr, g.data(), sizeof(int32_t) * P * k);
    if (boundary && e == hipSuccess) {
        if (hipMalloc((void **)&c->d_bnd, P) != hipSuccess) e = hipErrorOutOfMemory;
        cp(c->d_bnd, boundary, P);
    }
    if (e == hipSuccess)
        e = launch_setup_points(d_pos, d_vel, c->d_nh2, c->d_T, d_vt, d_X, c->mass, P, c->d_cell, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(d_pos);
    dfree(d_vel);
    dfree(d_vt);
    dfree(d_X);
    if (e != hipSuccess) return fail(c, NLTE_E_HIP, std::string("model upload: ") + hipGetErrorString(e));
    c->P = P;
    c->k = k;
    c->n_models = n_models;
    c->offsets = off;
    c->have_model = true;
    c->traced = false;
    c->scat_on = false;     // scattering opacities belong to the previous points
    c->dip_on = false;
    c->jnu_last = -1;
    drop_graphs(c);
    // point -> model map and per-model convergence state
    std::vector<int32_t> mo(P);
    for (int m = 0; m < n_models; ++m)
        for (int64_t p = off[m]; p < off[m + 1]; ++p) mo[p] = m;
    nlte_status st2;
    if ((st2 = dalloc(c, &c->d_model_of, P)) || (st2 = dalloc(c, &c->d_model_done, n_models)) ||
        (st2 = dalloc(c, &c->d_model_change, n_models)) || (st2 = dalloc(c, &c->d_model_iters, n_models)) ||
        (st2 = dalloc(c, &c->d_model_last, n_models)) || (st2 = dalloc(c, &c->d_model_off, n_models + 1)))
        return st2;
    HIPCHK(c, hipMemcpy(c->d_model_of, mo.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_model_off, off.data(), sizeof(int64_t) * (n_models + 1), hipMemcpyHostToDevice));
    // Morton processing order within each model (bounding box per model)
    {
        std::vector<double> box(6 * (size_t)n_models);
        for (int m = 0; m < n_models; ++m) {
            double lo[3], hi[3];
            for (int d = 0; d < 3; ++d) lo[d] = hi[d] = off[m] < off[m + 1] ? pos[3 * off[m] + d] : 0.0;
            for (int64_t p = off[m]; p < off[m + 1]; ++p)
                for (int d = 0; d < 3; ++d) {
                    lo[d] = std::min(lo[d], pos[3 * p + d]);
                    hi[d] = std::max(hi[d], pos[3 * p + d]);
                }
            for (int d = 0; d < 3; ++d) {
                box[6 * m + d] = lo[d];
                box[6 * m + 3 + d] = hi[d] - lo[d];
            }
        }
        double *d_box = nullptr;
        if ((st2 = dalloc(c, &d_box, box.size()))) return st2;
        if ((st2 = dalloc(c, &c->d_morton, P))) {
            dfree(d_box);
            return st2;
        }
        hipError_t e = hipMemcpy(d_box, box.data(), sizeof(double) * box.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = morton_order(c->d_cell, c->d_model_of, d_box, c->d_model_off, n_models, P, c->d_morton, c->stream);
        dfree(d_box);
        if (e != hipSuccess) return fail(c, NLTE_E_HIP, std::string("Morton order: ") + hipGetErrorString(e));
    }
    HIPCHK(c, hipMemset(c->d_model_done, 0, n_models));
    HIPCHK(c, hipMemset(c->d_model_iters, 0, sizeof(int32_t) * n_models));
    HIPCHK(c, hipMemset(c->d_model_last, 0, sizeof(double) * n_models));
    return ensure_work(c);
}

nlte_status nlte_set_rays(nlte_ctx *c, int n_rays, const double *dir)
{
    if (!c) return NLTE_E_INVALID_ARG;
    (void)hipSetDevice(c->device);
    if (n_rays < 2 || n_rays > 1024 || (n_rays & 1)) return fail(c, NLTE_E_INVALID_ARG, "n_rays must be even in [2, 1024]");
    if (!dir || !finite_all(dir, 3 * (int64_t)n_rays)) return fail(c, NLTE_E_INVALID_ARG, "bad directions");
    std::vector<int32_t> anti(n_rays, -1), pr;
    for (int r = 0; r < n_rays; ++r) {
        double nn = dir[3 * r] * dir[3 * r] + dir[3 * r + 1] * dir[3 * r + 1] + dir[3 * r + 2] * dir[3 * r + 2];
        if (fabs(nn - 1.0) > 1e-10) return fail(c, NLTE_E_INVALID_ARG, "directions must be unit vectors");
        for (int s = 0; s < n_rays; ++s) {
            double e = fabs(dir[3 * r] + dir[3 * s]) + fabs(dir[3 * r + 1] + dir[3 * s + 1]) +
                       fabs(dir[3 * r + 2] + dir[3 * s + 2]);
            if (e < 1e-12) {
                if (anti[r] >= 0) return fail(c, NLTE_E_INVALID_ARG, "duplicate antipodes");
                anti[r] = s;
            }
        }
        if (anti[r] < 0) return fail(c, NLTE_E_INVALID_ARG, "ray set is not point-symmetric");
    }
    for (int r = 0; r < n_rays; ++r)
        if (r < anti[r]) pr.push_back(r);
    nlte_status st;
    if ((st = dalloc(c, &c->d_dir, 3 * (size_t)n_rays)) || (st = dalloc(c, &c->d_anti, n_rays)) ||
        (st = dalloc(c, &c->d_pair_r, pr.size())))
        return st;
    HIPCHK(c, hipMemcpy(c->d_dir, dir, sizeof(double) * 3 * n_rays, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_anti, anti.data(), sizeof(int32_t) * n_rays, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_pair_r, pr.data(), sizeof(int32_t) * pr.size(), hipMemcpyHostToDevice));
    c->n_rays = n_rays;
    c->n_pairs = (int)pr.size();
    c->anti = anti;
    c->pair_r = pr;
    c->dir_host.assign(dir, dir + 3 * (size_t)n_rays);
    c->have_rays = true;
    c->traced = false;
    drop_graphs(c);
    return NLTE_OK;
}

nlte_status nlte_set_rays_healpix(nlte_ctx *c, int nside)
{
    if (!c) return NLTE_E_INVALID_ARG;
    if (nside < 1 || 12 * nside * nside > 1024) return fail(c, NLTE_E_INVALID_ARG, "nside must be in 1..9");
    // HEALPix RING pixel centres (Gorski et al. 2005), ring by ring from the north pole;
    // within a ring by increasing azimuth, starting where the RING scheme numbers it
    const int N = nside;
    const double pi = 3.14159265358979323846;
    std::vector<double> dir;
    dir.reserve(3 * (size_t)12 * N * N);
    auto push = [&](double z, double phi) {
        const double st = sqrt(fmax(0.0, (1.0 - z) * (1.0 + z)));
        dir.push_back(st * cos(phi));
        dir.push_back(st * sin(phi));
        dir.push_back(z);
    };
    for (int i = 1; i < 4 * N; ++i) {
        if (i < N) {                      // north polar cap: 4 i pixels
            const double z = 1.0 - (double)(i * i) / (3.0 * N * N);
            for (int j = 1; j <= 4 * i; ++j) push(z, (j - 0.5) * (0.5 * pi) / i);
        } else if (i <= 3 * N) {          // equatorial belt: 4 N pixels, every other ring offset by half
            const double z = (2 * N - i) * 2.0 / (3.0 * N);
            const double shift = ((i + N) & 1) ? 1.0 : 0.5;
            for (int j = 1; j <= 4 * N; ++j) push(z, (j - shift) * pi / (2.0 * N));
        } else {                          // south polar cap, k-th ring from the south pole
            const int k = 4 * N - i;
            const double z = -1.0 + (double)(k * k) / (3.0 * N * N);
            for (int j = 1; j <= 4 * k; ++j) push(z, (j - 0.5) * (0.5 * pi) / k);
        }
    }
    return nlte_set_rays(c, (int)(dir.size() / 3), dir.data());
}

nlte_status nlte_get_rays(nlte_ctx *c, int *n_rays, double *dir)
{
    if (!c) return NLTE_E_INVALID_ARG;
    if (!c->have_rays) return fail(c, NLTE_E_STATE, "no rays have been set");
    if (n_rays) *n_rays = c->n_rays;
    if (dir) memcpy(dir, c->dir_host.data(), sizeof(double) * c->dir_host.size());
    return NLTE_OK;
}

nlte_status nlte_set_quadrature(nlte_ctx *c, int n_q, const double *x, const double *w)
{
    if (!c) return NLTE_E_INVALID_ARG;
    (void)hipSetDevice(c->device);
    if (n_q < 1 || n_q > 256 || !x || !w) return fail(c, NLTE_E_INVALID_ARG, "n_q out of [1, 256]");
    if (!finite_all(x, n_q) || !finite_all(w, n_q)) return fail(c, NLTE_E_INVALID_ARG, "non-finite quadrature");
    double sw = 0.0;
    for (int n = 0; n < n_q; ++n) {
        if (fabs(x[n] + x[n_q - 1 - n]) > 1e-12 || fabs(w[n] - w[n_q - 1 - n]) > 1e-12 || w[n] < 0.0)
            return fail(c, NLTE_E_INVALID_ARG, "quadrature must be symmetric with w >= 0");
        sw += w[n];
    }
    if (fabs(sw - 1.0) > 1e-12) return fail(c, NLTE_E_INVALID_ARG, "quadrature weights must sum to 1");
    nlte_status st;
    if ((st = dalloc(c, &c->d_qx, n_q)) || (st = dalloc(c, &c->d_qw, n_q))) return st;
    HIPCHK(c, hipMemcpy(c->d_qx, x, sizeof(double) * n_q, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_qw, w, sizeof(double) * n_q, hipMemcpyHostToDevice));
    c->n_q = n_q;
    c->xq_max = 0.0;
    for (int n = 0; n < n_q; ++n) c->xq_max = std::max(c->xq_max, fabs(x[n]));
    c->q_ascending = true;
    for (int n = 0; n + 1 < n_q; ++n)
        if (!(x[n] < x[n + 1])) c->q_ascending = false;
    // offsets evenly spaced to 1e-12 of the spacing let the scattering solve locate an
    // offset by its arithmetic position on the grid; other grids are searched by bisection
    c->q_uniform = false;
    if (c->q_ascending && n_q > 1) {
        const double h = (x[n_q - 1] - x[0]) / (double)(n_q - 1);
        bool even = true;
        for (int n = 0; n < n_q; ++n)
            if (fabs(x[n] - (x[0] + n * h)) > 1e-12 * h) even = false;
        c->q_uniform = even;
        c->q_inv_h = 1.0 / h;
    }
    c->have_quad = true;
    c->jnu_last = -1;
    drop_graphs(c);
    return NLTE_OK;
}

nlte_status nlte_set_params(nlte_ctx *c, const nlte_params *p)
{
    if (!c || !p) return NLTE_E_INVALID_ARG;
    if (!(p->t_cmb > 0.0) || !(p->f_sub > 0.0) || !(p->tol >= 0.0) || p->max_iter < 1 ||
        p->max_iter > 100000 || (p->precision != NLTE_PREC_FP64 && p->precision != NLTE_PREC_FP32_BULK) ||
        p->lines_per_lane < 0 || p->lines_per_lane > kMaxLpl || p->waves_per_simd < 0 ||
        p->waves_per_simd > 3 || p->long_segments < -1 || p->long_segments > 1 ||
        !(p->stage_nodes == 0 || (p->stage_nodes >= 2 && p->stage_nodes <= kWave)) || p->tile_points < 0 ||
        p->tile_points > 16 ||
        !(p->ng_every == 0 || (p->ng_every >= 3 && p->ng_every <= kNgMaxM)) ||
        !(p->alo_band == 0 || (p->alo_band == 1 && p->use_alo)))
        return fail(c, NLTE_E_INVALID_ARG,
                    "parameter out of range (lines_per_lane: 0..5; waves_per_simd: 0..3; long_segments: -1..1; "
                    "stage_nodes: 0 or 2..64; tile_points: 0..16; ng_every: 0 or 3..8; "
                    "alo_band: 0, or 1 with use_alo)");
    c->params = *p;
    c->cfg.lpl = p->lines_per_lane;
    c->cfg.waves = p->waves_per_simd;
    c->cfg.long_seg = p->long_segments;
    c->cfg.ns = p->stage_nodes;
    c->cfg.tile = p->tile_points;
    c->cfg.persistent = p->persistent ? 1 : 0;
    drop_graphs(c);
    return upload_ibdy(c);
}

nlte_status nlte_trace(nlte_ctx *c)
{
    nlte_status st = need(c, false);
    if (st) return st;
    (void)hipSetDevice(c->device);
    const int64_t n = c->P * c->n_rays;
    if ((st = dalloc(c, &c->d_roff, n + 1))) return st;
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemsetAsync(c->d_roff, 0, sizeof(int64_t), s));
    auto t0 = std::chrono::steady_clock::now();
    // neighbour slots with their positions, for the walks only (freed on every return)
    struct TabGuard {
        NbrEntry *p = nullptr;
        ~TabGuard() { dfree(p); }
    } tab;
    if ((st = dalloc(c, &tab.p, (size_t)(c->P * c->k)))) return st;
    HIPCHK(c, launch_nbr_table(c->d_cell, c->d_nbr, c->k, c->P, tab.p, s));
    HIPCHK(c, launch_walk_count(c->d_cell, tab.p, c->k, c->d_bnd, c->d_dir, c->n_rays, c->P,
                                c->d_roff + 1, s));
    size_t tmp_bytes = 0;
    HIPCHK(c, scan_lengths(c->d_roff, n, nullptr, &tmp_bytes, s));
    void *tmp = nullptr;
    HIPCHK(c, hipMalloc(&tmp, tmp_bytes ? tmp_bytes : 1));
    hipError_t e = scan_lengths(c->d_roff, n, tmp, &tmp_bytes, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    if (e != hipSuccess) return fail(c, NLTE_E_HIP, std::string("scan: ") + hipGetErrorString(e));
    int64_t total = 0;
    HIPCHK(c, hipMemcpy(&total, c->d_roff + n, sizeof(int64_t), hipMemcpyDeviceToHost));
    if ((st = dalloc(c, &c->d_rcells, (size_t)total))) return st;
    HIPCHK(c, launch_walk_fill(c->d_cell, tab.p, c->k, c->d_bnd, c->d_dir, c->n_rays, c->P,
                               c->d_roff, c->d_rcells, s));
    HIPCHK(c, hipStreamSynchronize(s));
    dfree(tab.p);
    auto t1 = std::chrono::steady_clock::now();
    c->st_trace.ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
    c->st_trace.launches += 1;
    // longest ray
    std::vector<int64_t> off(n + 1);
    HIPCHK(c, hipMemcpy(off.data(), c->d_roff, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    int mx = 0;
    for (int64_t i = 0; i < n; ++i) mx = std::max<int>(mx, (int)(off[i + 1] - off[i]));
    c->total_cells = total;
    c->max_len = mx;
    // elimination steps per frequency (cells + velocity sub-steps), per-point cost and
    // the points in decreasing-cost order for the persistent formal solve
    if ((st = dalloc(c, &c->d_cost, c->P))) return st;
    if ((st = dalloc(c, &c->d_order, c->P))) return st;
    unsigned long long *cost = c->d_cost;
    hipError_t e2 = hipMemsetAsync(cost, 0, sizeof(unsigned long long) * c->P, s);
    if (e2 == hipSuccess) e2 = hipMemsetAsync(c->d_maser, 0, sizeof(int64_t), s);
    SolveArgs a = solve_args(c, nullptr, nullptr, nullptr);
    if (e2 == hipSuccess) e2 = launch_count_steps(a, c->d_maser, cost, s);
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(&c->total_steps, c->d_maser, sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e2 == hipSuccess) e2 = sort_by_cost(cost, c->d_order, c->P, s);
    if (e2 != hipSuccess) return fail(c, NLTE_E_HIP, std::string("step count: ") + hipGetErrorString(e2));
    drop_graphs(c);
    c->traced = true;
    c->first_valid = false;
    return NLTE_OK;
}

nlte_status nlte_get_ray(nlte_ctx *c, int64_t point, int ray, int32_t *cells, int cap, int *len)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (point < 0 || point >= c->P || ray < 0 || ray >= c->n_rays || cap < 0 || (cap > 0 && !cells))
        return fail(c, NLTE_E_INVALID_ARG, "point or ray out of range");
    int64_t q = point * c->n_rays + ray, o[2];
    HIPCHK(c, hipMemcpy(o, c->d_roff + q, sizeof(int64_t) * 2, hipMemcpyDeviceToHost));
    int L = (int)(o[1] - o[0]);
    if (len) *len = L;
    int ncopy = std::min(L, cap);
    if (ncopy > 0) {
        HIPCHK(c, hipMemcpy(cells, c->d_rcells + o[0], sizeof(int32_t) * ncopy, hipMemcpyDeviceToHost));
        // model-local indices
        int m = (int)(std::upper_bound(c->offsets.begin(), c->offsets.end(), point) - c->offsets.begin()) - 1;
        for (int i = 0; i < ncopy; ++i) cells[i] -= (int32_t)c->offsets[m];
    }
    return NLTE_OK;
}

nlte_status nlte_get_order(nlte_ctx *c, int64_t *perm)
{
    if (!c) return NLTE_E_INVALID_ARG;
    if (!c->have_model) return fail(c, NLTE_E_STATE, "nlte_set_models has not been called");
    if (!perm) return fail(c, NLTE_E_INVALID_ARG, "null output");
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<int32_t> o(c->P);
    HIPCHK(c, hipMemcpy(o.data(), c->d_morton, sizeof(int32_t) * c->P, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < c->P; ++i) perm[i] = o[i];
    return NLTE_OK;
}

nlte_status nlte_get_point_cost(nlte_ctx *c, int64_t *cost)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!cost) return fail(c, NLTE_E_INVALID_ARG, "null output");
    static_assert(sizeof(unsigned long long) == sizeof(int64_t), "cost element size");
    HIPCHK(c, hipMemcpy(cost, c->d_cost, sizeof(int64_t) * c->P, hipMemcpyDeviceToHost));
    return NLTE_OK;
}

nlte_status nlte_trace_stats(nlte_ctx *c, int64_t *total_cells, int *max_len, int64_t *total_steps)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (total_cells) *total_cells = c->total_cells;
    if (max_len) *max_len = c->max_len;
    if (total_steps) *total_steps = c->total_steps;
    return NLTE_OK;
}

nlte_status nlte_get_line_width_speed(nlte_ctx *c, double *vw)
{
    if (!c || !vw) return NLTE_E_INVALID_ARG;
    if (!c->have_model) return fail(c, NLTE_E_STATE, "no model");
    std::vector<CellRec> h(c->P);
    HIPCHK(c, hipMemcpy(h.data(), c->d_cell, sizeof(CellRec) * c->P, hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < c->P; ++p) vw[p] = h[p].vw;
    return NLTE_OK;
}

nlte_status nlte_lte_dev(nlte_ctx *c, double *d_pops, void *stream)
{
    nlte_status st = need(c, false);
    if (st) return st;
    if (!d_pops) return fail(c, NLTE_E_INVALID_ARG, "null pops");
    (void)hipSetDevice(c->device);
    hipStream_t s = pick(c, stream);
    HIPCHK(c, timed(c, c->st_lte, s, [&] { return launch_lte(c->sp, c->d_cell, c->d_T, c->P, d_pops, s); }));
    return NLTE_OK;
}

nlte_status nlte_lte(nlte_ctx *c, double *pops)
{
    if (!pops) return fail(c, NLTE_E_INVALID_ARG, "null pops");
    nlte_status st = nlte_lte_dev(c, c ? c->d_pops_a : nullptr, nullptr);
    if (st) return st;
    HIPCHK(c, hipMemcpyAsync(pops, c->d_pops_a, sizeof(double) * c->P * c->n_lev, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NLTE_OK;
}

nlte_status nlte_formal_solve_dev(nlte_ctx *c, const double *d_pops, double *d_J, double *d_Jeff,
                                  double *d_L, void *stream)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!d_pops || !d_J || !d_Jeff || !d_L) return fail(c, NLTE_E_INVALID_ARG, "null buffer");
    (void)hipSetDevice(c->device);
    hipStream_t s = pick(c, stream);
    // a fill kernel, not a memset node: callers may capture this stream in a graph
    HIPCHK(c, launch_fill_u64(reinterpret_cast<unsigned long long *>(c->d_maser), 1, 0ull, s));
    return formal_solve_impl(c, d_pops, d_J, d_Jeff, d_L, s);
}

nlte_status nlte_formal_solve_noalloc_dev(nlte_ctx *c, const double *d_pops, double *d_J, double *d_Jeff,
                                          double *d_L, void *stream)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!d_pops || !d_J || !d_Jeff || !d_L) return fail(c, NLTE_E_INVALID_ARG, "null buffer");
    if (c->device < 0 || c->device >= kMaxDevices) return fail(c, NLTE_E_HIP, "device index beyond the scratch table");
    void *base = g_scratch_ptr[c->device];
    if (!base)
        return fail(c, NLTE_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(g_scratch_rc[c->device]));
    const size_t elem = c->params.precision == NLTE_PREC_FP32_BULK ? sizeof(float2) : sizeof(double2);
    const size_t need_bytes = (size_t)c->P * (size_t)c->n_lines * elem;
    if (need_bytes > kScratchBytes - kScratchHead)
        return fail(c, NLTE_E_INVALID_ARG,
                    "nlte_formal_solve_noalloc_dev: " + std::to_string(c->P) + " points x " +
                        std::to_string(c->n_lines) + " lines need " + std::to_string(need_bytes) +
                        " bytes of line-coefficient staging; the fixed scratch holds " +
                        std::to_string(kScratchBytes - kScratchHead) + " (use nlte_formal_solve_dev)");
    (void)hipSetDevice(c->device);
    hipStream_t s = pick(c, stream);
    FsScratch sc{static_cast<unsigned char *>(base) + kScratchHead, static_cast<unsigned long long *>(base)};
    // enqueue only: no event timing (which would synchronise), no step counting
    return formal_solve_impl(c, d_pops, d_J, d_Jeff, d_L, s, false, true, &sc);
}

nlte_status nlte_formal_solve(nlte_ctx *c, const double *pops, double *J, double *Jeff, double *L)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!pops || !J || !Jeff || !L) return fail(c, NLTE_E_INVALID_ARG, "null buffer");
    (void)hipSetDevice(c->device);
    const size_t np = sizeof(double) * c->P * c->n_lev, nj = sizeof(double) * c->P * c->n_lines;
    HIPCHK(c, hipMemcpyAsync(c->d_pops_a, pops, np, hipMemcpyHostToDevice, c->stream));
    if ((st = nlte_formal_solve_dev(c, c->d_pops_a, c->d_J, c->d_Jeff, c->d_L, nullptr))) return st;
    HIPCHK(c, hipMemcpyAsync(J, c->d_J, nj, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Jeff, c->d_Jeff, nj, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(L, c->d_L, nj, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NLTE_OK;
}

nlte_status nlte_stateq_dev(nlte_ctx *c, const double *d_old, const double *d_J, const double *d_Jeff,
                            const double *d_L, double *d_new, uint8_t *d_flags, void *stream)
{
    nlte_status st = need(c, false);
    if (st) return st;
    if (!d_old || !d_J || !d_Jeff || !d_L || !d_new) return fail(c, NLTE_E_INVALID_ARG, "null buffer");
    (void)hipSetDevice(c->device);
    return stateq_impl(c, d_old, d_J, d_Jeff, d_L, d_new, d_flags, nullptr, pick(c, stream));
}

nlte_status nlte_stateq(nlte_ctx *c, const double *pops_old, const double *J, const double *Jeff,
                        const double *L, double *pops_new, uint8_t *flags)
{
    nlte_status st = need(c, false);
    if (st) return st;
    if (!pops_old || !J || !Jeff || !L || !pops_new) return fail(c, NLTE_E_INVALID_ARG, "null buffer");
    (void)hipSetDevice(c->device);
    const size_t np = sizeof(double) * c->P * c->n_lev, nj = sizeof(double) * c->P * c->n_lines;
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemcpyAsync(c->d_pops_a, pops_old, np, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d_J, J, nj, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d_Jeff, Jeff, nj, hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(c->d_L, L, nj, hipMemcpyHostToDevice, s));
    if ((st = stateq_impl(c, c->d_pops_a, c->d_J, c->d_Jeff, c->d_L, c->d_pops_b, c->d_flags, nullptr, s)))
        return st;
    HIPCHK(c, hipMemcpyAsync(pops_new, c->d_pops_b, np, hipMemcpyDeviceToHost, s));
    if (flags) HIPCHK(c, hipMemcpyAsync(flags, c->d_flags, c->P, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return NLTE_OK;
}

nlte_status nlte_run_ali_dev(nlte_ctx *c, const double *d_init, double *d_out, nlte_ali_report *rep,
                             void *stream)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!d_out) return fail(c, NLTE_E_INVALID_ARG, "null output");
    (void)hipSetDevice(c->device);
    // the iterations run on the context's stream, ordered after the caller's stream
    hipStream_t s = c->stream;
    hipStream_t us = stream ? (hipStream_t)stream : c->stream;
    if (us != s) {
        HIPCHK(c, hipEventRecord(c->ev0, us));
        HIPCHK(c, hipStreamWaitEvent(s, c->ev0, 0));
    }
    const size_t np = sizeof(double) * c->P * c->n_lev;
    auto t0 = std::chrono::steady_clock::now();
    if (d_init)
        HIPCHK(c, hipMemcpyAsync(c->d_pops_a, d_init, np, hipMemcpyDeviceToDevice, s));
    else
        HIPCHK(c, launch_lte(c->sp, c->d_cell, c->d_T, c->P, c->d_pops_a, s));
    HIPCHK(c, launch_fill_u8(c->d_model_done, c->n_models, 0, s));
    HIPCHK(c, launch_fill_u8(reinterpret_cast<uint8_t *>(c->d_model_iters), sizeof(int32_t) * (int64_t)c->n_models, 0,
                             s));
    double *buf[2] = {c->d_pops_a, c->d_pops_b};
    const bool band = c->params.alo_band != 0;
    const bool scat = c->scat_on;
    if (band && scat) return fail(c, NLTE_E_INVALID_ARG, "the band ALO does not take scattering");
    if (band && (st = ensure_band(c))) return st;
    if (scat) {
        if ((st = need_scat(c)) || (st = ensure_jnu(c))) return st;
        HIPCHK(c, launch_jnu_start(c->d_ibdy, c->P, c->n_lines, c->n_q, c->d_jnu[0], s));
        c->jnu_last = 0;
    }
    const bool graph = c->params.use_graph != 0 && !c->params.profile && !band && !scat;
    if (graph) {
        if ((st = ensure_graph(c, 0, buf[0], buf[1]))) return st;
        if ((st = ensure_graph(c, 1, buf[1], buf[0]))) return st;
    }
    if (rep) memset(rep, 0, sizeof(*rep));
    const int M = c->params.ng_every;
    if (M > 0 && (st = ensure_ng(c))) return st;
    if (M > 0) HIPCHK(c, launch_fill_u64(c->d_ng_rej, 1, 0ull, s));
    const size_t nel = (size_t)c->P * c->n_lev;
    int it = 0, active = c->n_models, n_ng = 0, n_band = 0;
    ConvResult last{};
    while (it < c->params.max_iter) {
        const int slot = it & 1;
        if (band) {
            int used = 0;
            if ((st = iteration_band(c, buf[slot], buf[slot ^ 1], s, &used))) return st;
            n_band += used > 0;
        } else if (scat) {
            if ((st = iteration_scat(c, buf[slot], buf[slot ^ 1], s))) return st;
        } else if (graph)
            HIPCHK(c, hipGraphLaunch(c->graph_exec[slot], s));
        else if ((st = enqueue_iteration(c, buf[slot], buf[slot ^ 1], s, false)))
            return st;
        HIPCHK(c, hipStreamSynchronize(s));
        last = *c->h_conv;
        active = *c->h_active;
        if (rep && it < 1024) {
            rep->max_change[it] = last.max_change;
            rep->mean_change[it] = last.mean_change;
        }
        ++it;
        if (active == 0) break;
        if (M > 0) {
            // keep this iterate; after every M of them extrapolate (Sec. 3.4)
            double *newest = buf[it & 1];
            HIPCHK(c, hipMemcpyAsync(c->d_ng_hist + (size_t)((it - 1) % M) * nel, newest, sizeof(double) * nel,
                                     hipMemcpyDeviceToDevice, s));
            if (it % M == 0) {
                NgHist h{};
                h.M = M;
                for (int j = 0; j < M; ++j) h.x[j] = c->d_ng_hist + (size_t)((it - 1 - j) % M) * nel;
                HIPCHK(c, launch_ng(h, c->d_cell, c->d_model_off, c->d_model_done, c->d_model_of, c->n_models,
                                    c->n_lev, c->P, c->d_ng_part, c->d_ng_coef, c->d_ng_ok, newest, c->d_ng_rej, s));
                ++n_ng;
            }
        }
    }
    const double *cur = buf[it & 1];
    HIPCHK(c, hipMemcpyAsync(d_out, cur, np, hipMemcpyDeviceToDevice, s));
    int64_t maser = 0;
    HIPCHK(c, hipMemcpyAsync(&maser, c->d_maser, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    if (rep) {
        if (M > 0) {
            unsigned long long rej = 0;
            HIPCHK(c, hipMemcpy(&rej, c->d_ng_rej, sizeof(rej), hipMemcpyDeviceToHost));
            rep->n_ng_rejected = (int64_t)rej;
        }
        rep->n_ng_steps = n_ng;
        rep->n_band = n_band;
        rep->iterations = it;
        rep->converged = active == 0 ? 1 : 0;
        rep->n_models_converged = c->n_models - active;
        rep->n_fallback = last.n_fallback;
        rep->n_kept = last.n_kept;
        rep->n_maser = maser;
        rep->ms_total = std::chrono::duration<double, std::milli>(t1 - t0).count();
    }
    if (active != 0) {
        c->err = "ALI stopped at max_iter above tol";
        return NLTE_W_NOT_CONVERGED;
    }
    if (last.n_fallback || last.n_kept) {
        c->err = "some points fell back or kept their populations";
        return NLTE_W_NONPHYSICAL;
    }
    return NLTE_OK;
}

nlte_status nlte_run_ali(nlte_ctx *c, const double *pops_init, double *pops_out, nlte_ali_report *rep)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!pops_out) return fail(c, NLTE_E_INVALID_ARG, "null output");
    (void)hipSetDevice(c->device);
    const size_t np = sizeof(double) * c->P * c->n_lev;
    double *d_in = nullptr, *d_out = nullptr;
    if ((st = dalloc(c, &d_out, (size_t)c->P * c->n_lev))) return st;
    if (pops_init) {
        if ((st = dalloc(c, &d_in, (size_t)c->P * c->n_lev))) {
            dfree(d_out);
            return st;
        }
        if (hipMemcpy(d_in, pops_init, np, hipMemcpyHostToDevice) != hipSuccess) {
            dfree(d_in);
            dfree(d_out);
            return fail(c, NLTE_E_HIP, "copy of pops_init failed");
        }
    }
    nlte_status rs = nlte_run_ali_dev(c, d_in, d_out, rep, nullptr);
    if (rs >= 0) {
        if (hipMemcpy(pops_out, d_out, np, hipMemcpyDeviceToHost) != hipSuccess) rs = NLTE_E_HIP;
    }
    dfree(d_in);
    dfree(d_out);
    return rs;
}

nlte_status nlte_get_model_status(nlte_ctx *c, int32_t *iterations, uint8_t *converged, double *last_change)
{
    if (!c) return NLTE_E_INVALID_ARG;
    if (!c->have_model) return fail(c, NLTE_E_STATE, "no model");
    const int n = c->n_models;
    if (iterations) HIPCHK(c, hipMemcpy(iterations, c->d_model_iters, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    if (converged) HIPCHK(c, hipMemcpy(converged, c->d_model_done, n, hipMemcpyDeviceToHost));
    if (last_change) HIPCHK(c, hipMemcpy(last_change, c->d_model_last, sizeof(double) * n, hipMemcpyDeviceToHost));
    return NLTE_OK;
}

#ifndef NLTE_BUILD_ID
#define NLTE_BUILD_ID "unknown"
#endif

// Median time of `trials` formal-solve launches (after one warm-up) with launch choice k.
nlte_status time_choice(nlte_ctx *c, const SolveConfig &k, int trials, double *ms_out)
{
    hipStream_t s = c->stream;
    c->cfg = k;
    std::vector<float> t;
    for (int i = 0; i <= trials; ++i) {
        HIPCHK(c, hipEventRecord(c->ev0, s));
        nlte_status st = formal_solve_impl(c, c->d_pops_a, c->d_J, c->d_Jeff, c->d_L, s);
        if (st) return st;
        HIPCHK(c, hipEventRecord(c->ev1, s));
        HIPCHK(c, hipEventSynchronize(c->ev1));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
        if (i > 0) t.push_back(ms);
    }
    std::sort(t.begin(), t.end());
    *ms_out = t[t.size() / 2];
    return NLTE_OK;
}

nlte_status nlte_autotune(nlte_ctx *c, const char *cache_path, int trials, char *choice, int cap)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (trials < 1) trials = 3;
    (void)hipSetDevice(c->device);
    hipStream_t s = c->stream;
    // the library build is part of the key: choices timed on other kernels are not reused
    char key[512];
    snprintf(key, sizeof key, "%s|build=%s|P=%lld|rays=%d|lines=%d|nq=%d|steps=%lld|prec=%d",
             c->device_name.c_str(), NLTE_BUILD_ID, (long long)c->P, c->n_rays, c->n_lines, c->n_q,
             (long long)c->total_steps, c->params.precision);
    SolveConfig best = c->cfg;
    double best_ms = -1.0;
    bool cached = false;
    if (cache_path) {
        FILE *f = fopen(cache_path, "r");
        if (f) {
            char line[1024];
            while (fgets(line, sizeof line, f)) {
                char k2[512];
                int lpl, wv, far, ns, pe, tl;
                double ms;
                if (sscanf(line, "%511s lpl=%d waves=%d long=%d ns=%d persistent=%d tile=%d ms=%lf", k2, &lpl, &wv,
                           &far, &ns, &pe, &tl, &ms) == 8 &&
                    strcmp(k2, key) == 0) {
                    best.lpl = lpl;
                    best.waves = wv;
                    best.long_seg = far;
                    best.ns = ns;
                    best.persistent = pe;
                    best.tile = tl;
                    best_ms = ms;
                    cached = true;
                }
            }
            fclose(f);
        }
    }
    if (!cached) {
        HIPCHK(c, launch_lte(c->sp, c->d_cell, c->d_T, c->P, c->d_pops_a, s));
        const int saved_profile = c->params.profile;
        c->params.profile = 0;
        const SolveConfig saved = c->cfg;
        // the rule's choice, made explicit, is the starting point
        SolveArgs a0 = solve_args(c, nullptr, nullptr, nullptr);
        SolveConfig cur = saved;
        cur.lpl = a0.lines_per_wave / a0.ngrp;
        cur.waves = a0.waves;
        cur.long_seg = a0.collapse;
        cur.ns = a0.ns;
        cur.tile = a0.tile;
        auto restore = [&](nlte_status code) {
            c->cfg = saved;
            c->params.profile = saved_profile;
            return code;
        };
        if ((st = time_choice(c, cur, trials, &best_ms))) return restore(st);
        best = cur;
        const int lpl_cap = std::min(kMaxLpl, (c->n_lines + a0.ngrp - 1) / a0.ngrp);
        for (int dim = 0; dim < 6; ++dim) {
            std::vector<int> cand;
            if (dim == 0)
                for (int v = 1; v <= lpl_cap; ++v) cand.push_back(v);
            else if (dim == 1)
                cand = {1, 2, 3};
            else if (dim == 2)
                cand = {0, 1};
            else if (dim == 3)
                cand = {16, 32, 48, 64};
            else if (dim == 4)
                cand = {0, 1};
            else
                cand = {1, 2, 4, 8};
            for (int v : cand) {
                SolveConfig k = best;
                int *field = dim == 0   ? &k.lpl
                             : dim == 1 ? &k.waves
                             : dim == 2 ? &k.long_seg
                             : dim == 3 ? &k.ns
                             : dim == 4 ? &k.persistent
                                        : &k.tile;
                if (*field == v) continue;
                *field = v;
                if (dim == 0) k.ns = 0;   // a new line count takes the rule's staging depth
                double ms = 0.0;
                if ((st = time_choice(c, k, trials, &ms))) return restore(st);
                if (ms < best_ms) {
                    best_ms = ms;
                    best = k;
                }
            }
            if (dim == 0 && best.ns == 0) {   // make the staging depth explicit again
                c->cfg = best;
                SolveArgs ab = solve_args(c, nullptr, nullptr, nullptr);
                best.ns = ab.ns;
            }
        }
        restore(NLTE_OK);
        if (cache_path) {
            FILE *f = fopen(cache_path, "a");
            if (f) {
                fprintf(f, "%s lpl=%d waves=%d long=%d ns=%d persistent=%d tile=%d ms=%.4f\n", key, best.lpl,
                        best.waves, best.long_seg, best.ns, best.persistent, best.tile, best_ms);
                fclose(f);
            }
        }
    }
    c->cfg.lpl = best.lpl;
    c->cfg.waves = best.waves;
    c->cfg.long_seg = best.long_seg;
    c->cfg.ns = best.ns;
    c->cfg.persistent = best.persistent;
    c->cfg.tile = best.tile;
    c->params.lines_per_lane = best.lpl;
    c->params.waves_per_simd = best.waves;
    c->params.long_segments = best.long_seg;
    c->params.stage_nodes = best.ns;
    c->params.persistent = best.persistent;
    c->params.tile_points = best.tile;
    drop_graphs(c);
    if (choice && cap > 0)
        snprintf(choice, cap, "lpl=%d waves=%d long=%d ns=%d persistent=%d tile=%d ms=%.4f%s", best.lpl, best.waves,
                 best.long_seg, best.ns, best.persistent, best.tile, best_ms, cached ? " (cached)" : "");
    return NLTE_OK;
}

nlte_status nlte_get_launch(nlte_ctx *c, int *lines_per_lane, int *waves_per_simd, int *long_segments, int *stage_nodes,
                            int *persistent, int *tile_points)
{
    nlte_status st = need(c, true);
    if (st) return st;
    const SolveArgs a = solve_args(c, nullptr, nullptr, nullptr);
    if (lines_per_lane) *lines_per_lane = a.lines_per_wave / a.ngrp;
    if (waves_per_simd) *waves_per_simd = a.waves;
    if (long_segments) *long_segments = a.collapse;
    if (stage_nodes) *stage_nodes = a.ns;
    if (persistent) *persistent = a.persistent;
    if (tile_points) *tile_points = a.tile;
    return NLTE_OK;
}

nlte_status nlte_kernel_stats(nlte_ctx *c, const char *name, double *ms, int64_t *launches)
{
    if (!c || !name) return NLTE_E_INVALID_ARG;
    KernelStat *k = nullptr;
    if (!strcmp(name, "line_coef")) k = &c->st_line_coef;
    else if (!strcmp(name, "formal_solve")) k = &c->st_formal;
    else if (!strcmp(name, "stateq")) k = &c->st_stateq;
    else if (!strcmp(name, "lte")) k = &c->st_lte;
    else if (!strcmp(name, "trace")) k = &c->st_trace;
    else if (!strcmp(name, "features")) k = &c->st_features;
    else if (!strcmp(name, "mlp_forward")) k = &c->st_mlp_forward;
    else if (!strcmp(name, "mlp_train")) k = &c->st_mlp_train;
    else if (!strcmp(name, "mlp_update")) k = &c->st_mlp_update;
    else if (!strcmp(name, "image")) k = &c->st_image;
    if (!k) return fail(c, NLTE_E_INVALID_ARG, "unknown kernel name");
    if (ms) *ms = k->ms;
    if (launches) *launches = k->launches;
    return NLTE_OK;
}

nlte_status nlte_reset_kernel_stats(nlte_ctx *c)
{
    if (!c) return NLTE_E_INVALID_ARG;
    c->st_line_coef = c->st_formal = c->st_stateq = c->st_lte = c->st_trace = KernelStat{};
    c->st_features = c->st_mlp_forward = c->st_mlp_train = c->st_mlp_update = c->st_image = KernelStat{};
    if (c->d_exec) {
        (void)hipSetDevice(c->device);
        HIPCHK(c, hipDeviceSynchronize());
        HIPCHK(c, hipMemset(c->d_exec, 0, sizeof(unsigned long long)));
        HIPCHK(c, hipDeviceSynchronize());
    }
    return NLTE_OK;
}

nlte_status nlte_executed_steps(nlte_ctx *c, int64_t *node_freq)
{
    if (!c || !node_freq) return NLTE_E_INVALID_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipDeviceSynchronize());
    unsigned long long v = 0;
    HIPCHK(c, hipMemcpy(&v, c->d_exec, sizeof(v), hipMemcpyDeviceToHost));
    *node_freq = (int64_t)v;
    return NLTE_OK;
}


// ------------------------------------------------------------------ warm start

void nlte_default_train_params(nlte_train_params *p)
{
    if (!p) return;
    p->steps = 1000;
    p->batch = 4096;
    p->lr = 1e-3;
    p->beta1 = 0.9;
    p->beta2 = 0.999;
    p->eps = 1e-8;
}

int64_t nlte_mlp_param_count(int n_out)
{
    if (n_out < 1 || n_out > kMaxLev) return -1;
    return mlp_dims(n_out).n_params;
}

nlte_status nlte_features_dev(nlte_ctx *c, double *d_F, void *stream)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!d_F) return fail(c, NLTE_E_INVALID_ARG, "null output");
    HIPCHK(c, hipSetDevice(c->device));
    return features_impl(c, d_F, pick(c, stream));
}

nlte_status nlte_features(nlte_ctx *c, double *F)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!F) return fail(c, NLTE_E_INVALID_ARG, "null output");
    HIPCHK(c, hipSetDevice(c->device));
    double *d = nullptr;
    if ((st = dalloc(c, &d, (size_t)c->P * 8))) return st;
    st = features_impl(c, d, c->stream);
    hipError_t e = hipSuccess;
    if (!st) e = hipMemcpyAsync(F, d, sizeof(double) * c->P * 8, hipMemcpyDeviceToHost, c->stream);
    if (!st && e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(d);
    if (st) return st;
    if (e != hipSuccess) return fail(c, NLTE_E_HIP, std::string("features copy: ") + hipGetErrorString(e));
    return NLTE_OK;
}

nlte_status nlte_mlp_init(nlte_ctx *c, int n_out, uint64_t seed)
{
    if (!c) return NLTE_E_INVALID_ARG;
    HIPCHK(c, hipSetDevice(c->device));
    nlte_status st = mlp_alloc(c, n_out);
    if (st) return st;
    const MlpDims &d = c->mlp.dims;
    std::vector<float> theta(d.n_params, 0.0f);
    uint64_t state = seed;
    for (int l = 0; l < 4; ++l) {
        const double a = sqrt(6.0 / (double)(d.in[l] + d.out[l]));
        for (int64_t i = 0; i < (int64_t)d.in[l] * d.out[l]; ++i) {
            const double u = (double)(splitmix64(state) >> 11) * 0x1.0p-53;
            theta[d.w_off[l] + i] = (float)(a * (2.0 * u - 1.0));
        }
    }
    return mlp_upload(c, theta);
}

nlte_status nlte_mlp_set_weights(nlte_ctx *c, int n_out, const float *theta)
{
    if (!c) return NLTE_E_INVALID_ARG;
    if (!theta) return fail(c, NLTE_E_INVALID_ARG, "null weights");
    if (n_out < 1 || n_out > kMaxLev) return fail(c, NLTE_E_INVALID_ARG, "n_out must be in 1..16");
    const int64_t np = mlp_dims(n_out).n_params;
    std::vector<float> t(theta, theta + np);
    for (int64_t i = 0; i < np; ++i)
        if (!std::isfinite(t[i])) return fail(c, NLTE_E_INVALID_ARG, "non-finite weight");
    HIPCHK(c, hipSetDevice(c->device));
    nlte_status st = mlp_alloc(c, n_out);
    if (st) return st;
    return mlp_upload(c, t);
}

nlte_status nlte_mlp_get_weights(nlte_ctx *c, float *theta)
{
    nlte_status st = need_mlp(c);
    if (st) return st;
    if (!theta) return fail(c, NLTE_E_INVALID_ARG, "null output");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(theta, c->mlp.d_theta, sizeof(float) * c->mlp.dims.n_params, hipMemcpyDeviceToHost));
    return NLTE_OK;
}

nlte_status nlte_mlp_set_norm(nlte_ctx *c, const double *mean, const double *std)
{
    if (!c) return NLTE_E_INVALID_ARG;
    if (!mean || !std) return fail(c, NLTE_E_INVALID_ARG, "null mean or std");
    for (int f = 0; f < 8; ++f)
        if (!std::isfinite(mean[f]) || !std::isfinite(std[f]) || !(std[f] > 0.0))
            return fail(c, NLTE_E_INVALID_ARG, "mean must be finite and std finite and positive");
    for (int f = 0; f < 8; ++f) {
        c->mlp.norm.mean[f] = mean[f];
        c->mlp.norm.std[f] = std[f];
    }
    return NLTE_OK;
}

nlte_status nlte_mlp_forward(nlte_ctx *c, const float *X, int64_t n, float *Y)
{
    nlte_status st = need_mlp(c);
    if (st) return st;
    if (n < 0 || (n > 0 && (!X || !Y))) return fail(c, NLTE_E_INVALID_ARG, "invalid rows");
    if (n == 0) return NLTE_OK;
    HIPCHK(c, hipSetDevice(c->device));
    if ((st = mlp_ensure_rows(c, n))) return st;
    MlpState &m = c->mlp;
    const int no = m.dims.out[3];
    HIPCHK(c, hipMemcpyAsync(m.d_x, X, sizeof(float) * n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_mlp_forward(m.d_frags, m.d_theta, m.dims, m.d_x, n, m.d_y, c->stream));
    HIPCHK(c, hipMemcpyAsync(Y, m.d_y, sizeof(float) * n * no, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NLTE_OK;
}

nlte_status nlte_mlp_loss_grad(nlte_ctx *c, const float *X, const float *T, int64_t n, float *grad, double *loss)
{
    nlte_status st = need_mlp(c);
    if (st) return st;
    if (n < 1 || n > kMlpMaxRows || !X || !T) return fail(c, NLTE_E_INVALID_ARG, "invalid rows (1..65536)");
    HIPCHK(c, hipSetDevice(c->device));
    MlpState &m = c->mlp;
    const int no = m.dims.out[3];
    if ((st = mlp_ensure_rows(c, n))) return st;
    if ((st = mlp_ensure_batch(c, (int)n))) return st;
    if (!m.d_loss && (st = dalloc(c, &m.d_loss, 1))) return st;
    if (m.loss_cap < 1) m.loss_cap = 1;
    HIPCHK(c, hipMemcpyAsync(m.d_x, X, sizeof(float) * n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(m.d_y, T, sizeof(float) * n * no, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, launch_mlp_train(m.d_frags, m.d_theta, m.dims, m.d_x, m.d_y, n, 0, (int)n, m.d_ht, m.d_dzt,
                               m.d_gpart, m.d_lpart,
                               c->stream));
    HIPCHK(c, launch_mlp_update(m.d_theta, m.d_m, m.d_v, m.d_frags, m.dims, m.d_gpart, (int)n, 0, 0.f, 0.f, 0.f,
                                0.f, 1.f, 1.f, m.d_lpart, (float)(1.0 / ((double)n * no)), m.d_loss, m.d_grad,
                                c->stream));
    float lval = 0.f;
    if (grad)
        HIPCHK(c, hipMemcpyAsync(grad, m.d_grad, sizeof(float) * m.dims.n_params, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&lval, m.d_loss, sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (loss) *loss = lval;
    return NLTE_OK;
}

nlte_status nlte_mlp_train_dev(nlte_ctx *c, const float *d_X, const float *d_T, int64_t n,
                               const nlte_train_params *tp, float *d_loss_curve, void *stream)
{
    nlte_status st = need_mlp(c);
    if (st) return st;
    if ((st = check_train_params(c, n, tp))) return st;
    if (!d_X || !d_T) return fail(c, NLTE_E_INVALID_ARG, "null rows");
    HIPCHK(c, hipSetDevice(c->device));
    return train_impl(c, d_X, d_T, n, tp, d_loss_curve, pick(c, stream));
}

nlte_status nlte_mlp_train(nlte_ctx *c, const float *X, const float *T, int64_t n, const nlte_train_params *tp,
                           float *loss_curve)
{
    nlte_status st = need_mlp(c);
    if (st) return st;
    if ((st = check_train_params(c, n, tp))) return st;
    if (!X || !T) return fail(c, NLTE_E_INVALID_ARG, "null rows");
    HIPCHK(c, hipSetDevice(c->device));
    MlpState &m = c->mlp;
    const int no = m.dims.out[3];
    if ((st = mlp_ensure_rows(c, n))) return st;
    if (tp->steps > m.loss_cap) {
        if ((st = dalloc(c, &m.d_loss, (size_t)tp->steps))) return st;
        m.loss_cap = tp->steps;
    }
    HIPCHK(c, hipMemcpyAsync(m.d_x, X, sizeof(float) * n * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(m.d_y, T, sizeof(float) * n * no, hipMemcpyHostToDevice, c->stream));
    if ((st = train_impl(c, m.d_x, m.d_y, n, tp, m.d_loss, c->stream))) return st;
    if (loss_curve && tp->steps > 0)
        HIPCHK(c, hipMemcpyAsync(loss_curve, m.d_loss, sizeof(float) * tp->steps, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NLTE_OK;
}

nlte_status nlte_mlp_predict_dev(nlte_ctx *c, double *d_pops, int64_t *n_fallback, void *stream)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if ((st = need_mlp(c))) return st;
    if (c->mlp.dims.out[3] != c->n_lev) return fail(c, NLTE_E_STATE, "network outputs differ from the level count");
    if (!d_pops) return fail(c, NLTE_E_INVALID_ARG, "null output");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick(c, stream);
    if ((st = predict_impl(c, d_pops, s))) return st;
    if (n_fallback) {
        unsigned long long bad = 0;
        HIPCHK(c, hipMemcpyAsync(&bad, c->mlp.d_bad, sizeof(bad), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipStreamSynchronize(s));
        *n_fallback = (int64_t)bad;
    }
    return NLTE_OK;
}

nlte_status nlte_mlp_predict(nlte_ctx *c, double *pops, int64_t *n_fallback)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!pops) return fail(c, NLTE_E_INVALID_ARG, "null output");
    if ((st = need_mlp(c))) return st;
    if (c->mlp.dims.out[3] != c->n_lev) return fail(c, NLTE_E_STATE, "network outputs differ from the level count");
    HIPCHK(c, hipSetDevice(c->device));
    if ((st = mlp_ensure_points(c))) return st;
    if ((st = predict_impl(c, c->mlp.d_pred, c->stream))) return st;
    unsigned long long bad = 0;
    HIPCHK(c, hipMemcpyAsync(pops, c->mlp.d_pred, sizeof(double) * c->P * c->n_lev, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&bad, c->mlp.d_bad, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (n_fallback) *n_fallback = (int64_t)bad;
    return NLTE_OK;
}

nlte_status nlte_mlp_rows_dev(nlte_ctx *c, const double *d_pops, float *d_X, float *d_T, void *stream)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!d_pops || !d_X || !d_T) return fail(c, NLTE_E_INVALID_ARG, "null pointer");
    HIPCHK(c, hipSetDevice(c->device));
    if ((st = mlp_ensure_points(c))) return st;
    hipStream_t s = pick(c, stream);
    if ((st = features_impl(c, c->mlp.d_feat, s))) return st;
    HIPCHK(c, launch_mlp_standardise(c->mlp.d_feat, c->mlp.norm, c->P, d_X, s));
    HIPCHK(c, launch_mlp_targets(c->sp, d_pops, c->d_cell, c->d_T, c->P, d_T, s));
    return NLTE_OK;
}

nlte_status nlte_run_ali_warm_dev(nlte_ctx *c, double *d_out, nlte_ali_report *rep, int *used_network, void *stream)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if ((st = need_mlp(c))) return st;
    if (c->mlp.dims.out[3] != c->n_lev) return fail(c, NLTE_E_STATE, "network outputs differ from the level count");
    if (!d_out) return fail(c, NLTE_E_INVALID_ARG, "null output");
    HIPCHK(c, hipSetDevice(c->device));
    if ((st = mlp_ensure_points(c))) return st;
    // the prediction runs on the caller's stream, which the ALI orders itself after
    hipStream_t us = pick(c, stream);
    if ((st = predict_impl(c, c->mlp.d_pred, us))) return st;
    st = nlte_run_ali_dev(c, c->mlp.d_pred, d_out, rep, us);
    if (used_network) *used_network = 1;
    if (st == NLTE_W_NOT_CONVERGED) {
        // the iteration did not settle from the predicted start: start again from LTE
        if (used_network) *used_network = 0;
        st = nlte_run_ali_dev(c, nullptr, d_out, rep, us);
    }
    return st;
}

nlte_status nlte_run_ali_warm(nlte_ctx *c, double *pops_out, nlte_ali_report *rep, int *used_network)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!pops_out) return fail(c, NLTE_E_INVALID_ARG, "null output");
    HIPCHK(c, hipSetDevice(c->device));
    double *d_out = nullptr;
    if ((st = dalloc(c, &d_out, (size_t)c->P * c->n_lev))) return st;
    nlte_status rs = nlte_run_ali_warm_dev(c, d_out, rep, used_network, nullptr);
    if (rs >= 0 && hipMemcpy(pops_out, d_out, sizeof(double) * c->P * c->n_lev, hipMemcpyDeviceToHost) != hipSuccess)
        rs = fail(c, NLTE_E_HIP, "copy of the populations failed");
    dfree(d_out);
    return rs;
}

// ------------------------------------------------------------------ scattering

nlte_status nlte_set_scattering(nlte_ctx *c, const double *chi_sca)
{
    if (!c) return NLTE_E_INVALID_ARG;
    if (!c->have_species) return fail(c, NLTE_E_STATE, "nlte_set_species has not been called");
    if (!c->have_model) return fail(c, NLTE_E_STATE, "nlte_set_models has not been called");
    (void)hipSetDevice(c->device);
    c->jnu_last = -1;
    c->dip_on = false;   // the odd part is bounded by the opacities it was set with
    if (!chi_sca) {
        c->scat_on = false;
        return NLTE_OK;
    }
    const int64_t n = c->P * c->n_lines;
    for (int64_t i = 0; i < n; ++i)
        if (!(chi_sca[i] >= 0.0) || !std::isfinite(chi_sca[i]))
            return fail(c, NLTE_E_INVALID_ARG, "scattering opacities must be finite and >= 0");
    nlte_status st;
    if ((st = dalloc(c, &c->d_chi_sca, (size_t)n))) return st;
    HIPCHK(c, hipMemcpy(c->d_chi_sca, chi_sca, sizeof(double) * n, hipMemcpyHostToDevice));
    c->scat_on = true;
    return NLTE_OK;
}

nlte_status nlte_set_scattering_dipole(nlte_ctx *c, const double *chi_dip)
{
    if (!c) return NLTE_E_INVALID_ARG;
    if (!c->scat_on) return fail(c, NLTE_E_STATE, "nlte_set_scattering has not been called");
    (void)hipSetDevice(c->device);
    c->jnu_last = -1;
    if (!chi_dip) {
        c->dip_on = false;
        return NLTE_OK;
    }
    const int64_t n = c->P * c->n_lines;
    std::vector<double> cs(n);
    HIPCHK(c, hipMemcpy(cs.data(), c->d_chi_sca, sizeof(double) * n, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < n; ++i) {
        const double *d = chi_dip + 3 * i;
        if (!std::isfinite(d[0]) || !std::isfinite(d[1]) || !std::isfinite(d[2]))
            return fail(c, NLTE_E_INVALID_ARG, "dipole scattering opacities must be finite");
        if (!(std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) <= cs[i] * (1.0 + 1e-12)))
            return fail(c, NLTE_E_INVALID_ARG,
                        "|chi_dip| exceeds chi_sca: the scattering opacity would be negative in some direction");
    }
    nlte_status st;
    if ((st = dalloc(c, &c->d_chi_dip, (size_t)(3 * n)))) return st;
    HIPCHK(c, hipMemcpy(c->d_chi_dip, chi_dip, sizeof(double) * 3 * n, hipMemcpyHostToDevice));
    c->dip_on = true;
    return NLTE_OK;
}

nlte_status nlte_formal_solve_scat_dev(nlte_ctx *c, const double *d_pops, const double *d_jnu_in, double *d_J,
                                       double *d_Jeff, double *d_L, double *d_jnu_out, void *stream)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if ((st = need_scat(c))) return st;
    if (!d_pops || !d_jnu_in || !d_J || !d_Jeff || !d_L || !d_jnu_out)
        return fail(c, NLTE_E_INVALID_ARG, "null buffer");
    if (d_jnu_in == d_jnu_out) return fail(c, NLTE_E_INVALID_ARG, "jnu_in and jnu_out must differ");
    (void)hipSetDevice(c->device);
    hipStream_t s = pick(c, stream);
    HIPCHK(c, launch_fill_u64(reinterpret_cast<unsigned long long *>(c->d_maser), 1, 0ull, s));
    return formal_solve_scat_impl(c, d_pops, d_jnu_in, d_J, d_Jeff, d_L, d_jnu_out, s, false);
}

nlte_status nlte_formal_solve_scat(nlte_ctx *c, const double *pops, const double *jnu_in, double *J, double *Jeff,
                                   double *Lstar, double *jnu_out)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if ((st = need_scat(c))) return st;
    if (!pops || !jnu_in || !J || !Jeff || !Lstar || !jnu_out) return fail(c, NLTE_E_INVALID_ARG, "null buffer");
    (void)hipSetDevice(c->device);
    if ((st = ensure_jnu(c))) return st;
    c->jnu_last = -1;   // the ALI's buffers are used as scratch here
    const size_t np = sizeof(double) * c->P * c->n_lev, nj = sizeof(double) * c->P * c->n_lines;
    const size_t nn = sizeof(double) * c->jnu_elems;
    HIPCHK(c, hipMemcpyAsync(c->d_pops_a, pops, np, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_jnu[0], jnu_in, nn, hipMemcpyHostToDevice, c->stream));
    if ((st = nlte_formal_solve_scat_dev(c, c->d_pops_a, c->d_jnu[0], c->d_J, c->d_Jeff, c->d_L, c->d_jnu[1],
                                         nullptr)))
        return st;
    HIPCHK(c, hipMemcpyAsync(J, c->d_J, nj, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Jeff, c->d_Jeff, nj, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Lstar, c->d_L, nj, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(jnu_out, c->d_jnu[1], nn, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NLTE_OK;
}

nlte_status nlte_scattering_field(nlte_ctx *c, double *jnu)
{
    if (!c) return NLTE_E_INVALID_ARG;
    if (!jnu) return fail(c, NLTE_E_INVALID_ARG, "null buffer");
    if (c->jnu_last < 0 || !c->d_jnu[c->jnu_last])
        return fail(c, NLTE_E_STATE, "no ALI with scattering has run since the last change of inputs");
    (void)hipSetDevice(c->device);
    HIPCHK(c, hipMemcpyAsync(jnu, c->d_jnu[c->jnu_last], sizeof(double) * c->jnu_elems, hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NLTE_OK;
}

// ------------------------------------------------------------------ band ALO

nlte_status nlte_formal_solve_band(nlte_ctx *c, const double *pops, double *J, double *Jeff, double *Lstar,
                                   double *Jb, double *Ld, double *Ln)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!pops || !J || !Jeff || !Lstar || !Jb || !Ld || !Ln) return fail(c, NLTE_E_INVALID_ARG, "null pointer");
    HIPCHK(c, hipSetDevice(c->device));
    if ((st = ensure_band(c))) return st;
    const size_t np = sizeof(double) * c->P * c->n_lev, nq = sizeof(double) * c->P * c->n_lines;
    HIPCHK(c, hipMemcpyAsync(c->d_pops_a, pops, np, hipMemcpyHostToDevice, c->stream));
    if ((st = formal_solve_band_impl(c, c->d_pops_a, c->d_J, c->d_Jeff, c->d_L, c->stream, false))) return st;
    HIPCHK(c, hipMemcpyAsync(J, c->d_J, nq, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Jeff, c->d_Jeff, nq, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Lstar, c->d_L, nq, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Jb, c->d_Jb, nq, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Ld, c->d_Ld, nq, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(Ln, c->d_Ln, nq * c->n_rays, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return NLTE_OK;
}

nlte_status nlte_stateq_band(nlte_ctx *c, const double *pops_old, const double *J, const double *Jeff,
                             const double *Lstar, const double *Jb, const double *Ld, const double *Ln,
                             double *pops_new, int *band_used, int *solver_iterations)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!pops_old || !J || !Jeff || !Lstar || !Jb || !Ld || !Ln || !pops_new)
        return fail(c, NLTE_E_INVALID_ARG, "null pointer");
    if (!c->params.use_alo) return fail(c, NLTE_E_STATE, "the band ALO needs use_alo = 1");
    HIPCHK(c, hipSetDevice(c->device));
    if ((st = ensure_band(c))) return st;
    const size_t np = sizeof(double) * c->P * c->n_lev, nq = sizeof(double) * c->P * c->n_lines;
    HIPCHK(c, hipMemcpyAsync(c->d_pops_a, pops_old, np, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_J, J, nq, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_Jeff, Jeff, nq, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_L, Lstar, nq, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_Jb, Jb, nq, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_Ld, Ld, nq, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_Ln, Ln, nq * c->n_rays, hipMemcpyHostToDevice, c->stream));
    int used = 0, iters = 0;
    if ((st = stateq_band_impl(c, c->d_pops_a, c->d_J, c->d_Jeff, c->d_L, c->d_pops_b, c->d_flags, c->stream, false,
                               &used, &iters)))
        return st;
    HIPCHK(c, hipMemcpyAsync(pops_new, c->d_pops_b, np, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (band_used) *band_used = used;
    if (solver_iterations) *solver_iterations = iters;
    return NLTE_OK;
}

// ------------------------------------------------------------------ imaging

nlte_status nlte_image_dev(nlte_ctx *c, const double *d_pops, int ray, int line, int n_ch, const double *v_ch,
                           double *d_I, double *d_xy, void *stream)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!d_pops || !d_I || !v_ch) return fail(c, NLTE_E_INVALID_ARG, "null pointer");
    if (ray < 0 || ray >= c->n_rays) return fail(c, NLTE_E_INVALID_ARG, "ray out of range");
    if (line < 0 || line >= c->n_lines) return fail(c, NLTE_E_INVALID_ARG, "line out of range");
    if (n_ch < 1 || n_ch > 1024) return fail(c, NLTE_E_INVALID_ARG, "n_ch must be in 1..1024");
    for (int i = 0; i < n_ch; ++i)
        if (!std::isfinite(v_ch[i])) return fail(c, NLTE_E_INVALID_ARG, "non-finite channel velocity");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t s = pick(c, stream);
    if (n_ch > c->vch_cap) {
        if ((st = dalloc(c, &c->d_vch, (size_t)n_ch))) return st;
        c->vch_cap = n_ch;
    }
    HIPCHK(c, hipMemcpyAsync(c->d_vch, v_ch, sizeof(double) * n_ch, hipMemcpyHostToDevice, s));
    // FP64 line coefficients of these populations
    HIPCHK(c, launch_line_coef(c->sp, c->d_cell, d_pops, c->P, 0, c->d_lc, c->d_maser, s));
    const double nu = c->nu[line];
    ImageArgs a{};
    a.cell = c->d_cell;
    a.lc = c->d_lc;
    a.roff = c->d_roff;
    a.rcells = c->d_rcells;
    a.dir = c->d_dir;
    a.anti = c->d_anti;
    a.v_ch = c->d_vch;
    a.I = d_I;
    a.f_sub = c->params.f_sub;
    a.I_in = 2.0 * kH * nu * nu * nu / (kC * kC) / expm1(kH * nu / (kKB * c->params.t_cmb));
    a.P = c->P;
    a.n_rays = c->n_rays;
    a.n_lines = c->n_lines;
    a.line = line;
    a.ray = ray;
    a.n_ch = n_ch;
    // image-plane basis: e1 = (z x n)/|z x n| (x-axis instead of z when |n_z| > 0.9), e2 = n x e1
    const double *dir = c->dir_host.data();
    const double n0 = dir[3 * ray], n1 = dir[3 * ray + 1], n2 = dir[3 * ray + 2];
    double r0 = 0.0, r1 = 0.0, r2 = 1.0;
    if (fabs(n2) > 0.9) {
        r0 = 1.0;
        r2 = 0.0;
    }
    double e1x = r1 * n2 - r2 * n1, e1y = r2 * n0 - r0 * n2, e1z = r0 * n1 - r1 * n0;
    const double en = sqrt(e1x * e1x + e1y * e1y + e1z * e1z);
    e1x /= en;
    e1y /= en;
    e1z /= en;
    const double3 e1 = make_double3(e1x, e1y, e1z);
    const double3 e2 = make_double3(n1 * e1z - n2 * e1y, n2 * e1x - n0 * e1z, n0 * e1y - n1 * e1x);
    HIPCHK(c, timed(c, c->st_image, s, [&] { return launch_image(a, s); }));
    if (d_xy) HIPCHK(c, launch_image_plane(c->d_cell, e1, e2, c->P, d_xy, s));
    return NLTE_OK;
}

nlte_status nlte_image(nlte_ctx *c, const double *pops, int ray, int line, int n_ch, const double *v_ch, double *I,
                       double *xy)
{
    nlte_status st = need(c, true);
    if (st) return st;
    if (!pops || !I) return fail(c, NLTE_E_INVALID_ARG, "null pointer");
    if (n_ch < 1 || n_ch > 1024) return fail(c, NLTE_E_INVALID_ARG, "n_ch must be in 1..1024");
    HIPCHK(c, hipSetDevice(c->device));
    double *d_I = nullptr, *d_xy = nullptr;
    if ((st = dalloc(c, &d_I, (size_t)c->P * n_ch))) return st;
    if (xy && (st = dalloc(c, &d_xy, (size_t)c->P * 2))) {
        dfree(d_I);
        return st;
    }
    hipError_t e = hipMemcpyAsync(c->d_pops_a, pops, sizeof(double) * c->P * c->n_lev, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) st = nlte_image_dev(c, c->d_pops_a, ray, line, n_ch, v_ch, d_I, d_xy, c->stream);
    if (e == hipSuccess && st == NLTE_OK)
        e = hipMemcpyAsync(I, d_I, sizeof(double) * c->P * n_ch, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && st == NLTE_OK && xy)
        e = hipMemcpyAsync(xy, d_xy, sizeof(double) * c->P * 2, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    dfree(d_I);
    dfree(d_xy);
    if (st) return st;
    if (e != hipSuccess) return fail(c, NLTE_E_HIP, std::string("image: ") + hipGetErrorString(e));
    return NLTE_OK;
}

}  // extern "C"
