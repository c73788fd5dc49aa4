// Internal declarations of the gfx950 library: device data layout, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "nlte.h"

namespace nlte {

// CGS constants (SI-exact values).
constexpr double kH = 6.62607015e-27;
constexpr double kKB = 1.380649e-16;
constexpr double kC = 2.99792458e10;
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;

constexpr int kMaxLev = 16;
constexpr int kMaxLines = 32;
constexpr int kWave = 64;
// Upper bound on the velocity sub-intervals of one segment (an implementation limit that
// keeps every sweep finite for any input; realistic models stay far below it).
constexpr int kMaxSub = 1 << 20;

// One gather-friendly 64-byte record per point: what a ray walk and a ray-pair sweep
// read from the cells they visit.
struct __align__(64) CellRec {
    double px, py, pz;  // position [cm]
    double vw;          // line-width speed sqrt(2kT/m + v_turb^2) [cm/s]
    double vx, vy, vz;  // velocity [cm/s]
    double ntot;        // species density abundance * n_H2 [cm^-3]
};

// Species tables in device memory (one allocation, pointers into it).
struct SpeciesDev {
    int n_lev, n_lines, n_coll, n_T;
    double mass;
    const int32_t *lu, *ll, *cu, *cl;
    const double *A, *nu, *Bul, *Blu, *pre;  // pre = h nu / 4 pi
    const double *E, *g, *Ttab, *Ktab;
};

// Per-iteration convergence partials written by the stat-eq kernel.
struct ConvPartial {
    double max_change;
    double sum_change;
    int64_t count;
    int64_t n_fallback;
    int64_t n_kept;
};

struct ConvResult {
    double max_change;
    double mean_change;
    int64_t n_fallback;
    int64_t n_kept;
};

struct SolveArgs {
    const CellRec *cell;
    const void *lc;          // [P][n_lines] (kappa, S): double2 (FP64) or float2 (FP32 bulk)
    const int64_t *roff;     // [P * n_rays + 1]
    const int32_t *rcells;   // cached walks, global point indices, nearest first
    const double *dir;       // [n_rays][3]
    const int32_t *pair_r;   // [n_pairs] representative ray of each pair
    const int32_t *anti;     // [n_rays]
    const double *qx, *qw;   // [n_q]
    const double *ibdy;      // [n_lines] boundary intensity
    double f_sub;
    double xq_max;           // max |x_q| of the quadrature
    double norm;             // 2 / n_rays
    int64_t P;
    int n_rays, n_pairs, n_q, n_lines;
    int groups;              // waves per point
    int lines_per_wave;      // lines one wave serves (lane groups x lines per lane)
    int ngrp;                // lane groups per wave (2 when 2 n_q <= 64, else 1)
    int fchunks;             // frequency chunks per wave (n_q > 64), else 1
    int ns;                  // ray nodes a wave stages in LDS per round (2..64)
    int waves;               // register budget of the launch: 2 or 3 waves per SIMD
    int collapse;            // 1: long-segment mode (profile recurrence, far-wing collapse)
    int persistent;          // 1: items from the work counter in decreasing-cost order
    int tile;                // work items a workgroup takes at a time (1..16)
    int64_t n_blocks;        // work items (P * groups)
    double *J, *Jeff, *L;    // [P][n_lines]
    double *Jb, *Ld;         // band operator: J without the band's share, its diagonal [P][n_lines]
    double *Ln;              // band operator: coupling to the first cell per ray [P][n_lines][n_rays]
    // ALI only: points of converged models are skipped (null: solve every point)
    const uint8_t *model_done;
    const int32_t *model_of;
    // persistent form: item order (points by decreasing cost) and the work counter
    const int32_t *order;
    unsigned long long *work_counter;
    // profile mode: executed node-frequency elimination steps (null: not counted)
    unsigned long long *exec_steps;
};

// Coupled statistical equilibrium of the band ALO (see band.hip).
struct BandArgs {
    const double *Jb, *Ld, *Ln;   // band formal-solve outputs
    const int32_t *first;         // [P][n_rays] first cell of each walk (-1: none)
    const uint8_t *done;          // converged models (held fixed; null: none)
    const int32_t *model_of;
    double *LU;                   // [P][n_lev][n_lev] factors of the points' own rate matrices
    int32_t *piv;                 // [P][n_lev]
    double *cpl;                  // [P][n_lines][n_rays] coupling coefficients
    double *x0;                   // [P][n_lev] uncoupled solution
    unsigned long long *bad;      // singular local matrices
    uint8_t *model_bad;           // [n_models] 1: the model takes the local solve this iteration
    int64_t P;
    int R;
};

struct DotArgs {
    const double *a[3];
    const double *b[3];
    int nd;
};

// Formal solve with scattering (see scatter.hip).
struct ScatArgs {
    const CellRec *cell;
    const void *lc;          // [P][n_lines] double2 (kappa, S), FP64
    const int64_t *roff;
    const int32_t *rcells;
    const double *dir;
    const int32_t *pair_r, *anti;
    const double *qx, *qw;   // [n_q], ascending and symmetric
    const double *ibdy;      // [n_lines]
    const double *chi_sca;   // [P][n_lines] scattering opacity chi^+ [cm^-1]
    const double *chi_dip;   // [P][n_lines][3] its odd part (chi^- = chi_dip . n), or null
    const double *Jin;       // [P][n_lines][n_q] previous weighted mean intensity Jw
    double *Jout;            // [P][n_lines][n_q]
    double *J, *Jeff, *L;    // [P][n_lines]
    double f_sub, norm, inv_rays;
    double q_inv_h;          // 1 / spacing of an evenly spaced quadrature
    int64_t P;
    int n_rays, n_pairs, n_q, n_lines;
    int q_uniform;           // 1: evenly spaced quadrature offsets
    const uint8_t *model_done;   // ALI only (null: solve every point)
    const int32_t *model_of;
};

// Image of the model along one ray direction (see image.hip).
struct ImageArgs {
    const CellRec *cell;
    const void *lc;          // [P][n_lines] double2 (kappa, S), FP64
    const int64_t *roff;
    const int32_t *rcells;
    const double *dir;
    const int32_t *anti;
    const double *v_ch;      // [n_ch] channel velocities [cm/s]
    double *I;               // [P][n_ch]
    double f_sub;
    double I_in;             // CMB intensity at the line centre
    int64_t P;
    int n_rays, n_lines, line, ray, n_ch;
};

// Ng acceleration: the last M iterates, newest first.
constexpr int kNgMaxM = 8;
constexpr int kNgMaxSums = (kNgMaxM - 2) * (kNgMaxM - 1) / 2 + (kNgMaxM - 2);
struct NgHist {
    const double *x[kNgMaxM];
    int M;
};

// Launch choices of the formal solve (picked by rule or by the autotuner).
constexpr int kMaxLpl = 5;    // lines per lane
struct SolveConfig {
    int lpl = 0;              // lines per lane (1..kMaxLpl; 0 = by rule)
    int waves = 0;            // register budget for 2 or 3 waves per SIMD (0 = by rule)
    int long_seg = -1;        // long-segment mode: 1 on, 0 off, -1 by the trace's steps per cell
    int ns = 0;               // ray nodes staged per round (2..64; 0 = by rule)
    int persistent = 0;       // 1: work-queue kernel in decreasing-cost order
    int tile = 0;             // work items per workgroup grab (1..16; 0 = 1)
    int n_wg = 0;             // workgroups of the persistent kernel
};

struct KernelStat {
    double ms = 0.0;
    int64_t launches = 0;
};

// Shapes of the warm-start network 8 -> 128 -> 128 -> 128 -> n_out and the offsets of
// each layer's weights and biases in the flat parameter vector.
struct MlpDims {
    int in[4], out[4];
    int64_t w_off[4], b_off[4];
    int64_t n_params;
};

// Feature standardisation (x - mean) / std; identity until set.
struct MlpNorm {
    double mean[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double std[8] = {1, 1, 1, 1, 1, 1, 1, 1};
};

// Parameters, optimiser state and work buffers of the warm-start network.
struct MlpState {
    bool ready = false;
    MlpDims dims{};
    MlpNorm norm{};
    int64_t step = 0;                 // Adam steps since init / set_weights
    float *d_theta = nullptr, *d_m = nullptr, *d_v = nullptr;  // [n_params]
    void *d_frags = nullptr;          // bfloat16 A operands packed from d_theta
    float *d_gpart = nullptr;         // [chunks][n_params] weight-gradient partials
    float *d_lpart = nullptr;         // [ld / 16] loss partials
    unsigned short *d_ht = nullptr;   // layer inputs of a batch (bfloat16, feature-major)
    float *d_dzt = nullptr;           // layer output gradients of a batch (feature-major)
    int64_t batch_cap = 0;            // largest batch the training buffers hold
    float *d_loss = nullptr;          // [loss_cap]
    int64_t loss_cap = 0;
    float *d_grad = nullptr;          // [n_params]
    float *d_x = nullptr, *d_y = nullptr;  // host-call staging: [rows][8], [rows][n_out]
    int64_t rows_cap = 0;
    double *d_feat = nullptr;         // [P][8]
    float *d_xp = nullptr, *d_yp = nullptr;  // [P][8], [P][n_out]
    double *d_pred = nullptr;         // [P][n_lev]
    int64_t pred_cap = 0;
    unsigned long long *d_bad = nullptr;
};

}  // namespace nlte

struct nlte_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    nlte_params params{};

    // species
    bool have_species = false;
    int n_lev = 0, n_lines = 0, n_coll = 0, n_T = 0;
    double mass = 0.0;
    std::vector<double> nu;  // host copy of line frequencies
    void *d_species_mem = nullptr;
    nlte::SpeciesDev sp{};

    // model(s)
    bool have_model = false;
    int64_t P = 0;
    int k = 0;
    int n_models = 0;
    std::vector<int64_t> offsets;   // [n_models + 1]
    int32_t *d_model_of = nullptr;  // [P]
    int64_t *d_model_off = nullptr; // [n_models + 1]
    int32_t *d_morton = nullptr;    // [P] points in Morton order within each model
    uint8_t *d_model_done = nullptr;            // [n_models]
    unsigned long long *d_model_change = nullptr;  // [n_models] max change as FP64 bits
    int32_t *d_model_iters = nullptr;           // [n_models]
    double *d_model_last = nullptr;             // [n_models]
    nlte::CellRec *d_cell = nullptr;
    double *d_nh2 = nullptr, *d_T = nullptr;
    int32_t *d_nbr = nullptr;  // global indices
    uint8_t *d_bnd = nullptr;

    // rays
    bool have_rays = false;
    int n_rays = 0, n_pairs = 0;
    std::vector<int32_t> pair_r, anti;
    double *d_dir = nullptr;
    int32_t *d_pair_r = nullptr, *d_anti = nullptr;

    // quadrature
    bool have_quad = false;
    int n_q = 0;
    double *d_qx = nullptr, *d_qw = nullptr;
    double *d_ibdy = nullptr;
    double xq_max = 0.0;

    // ray cache, per-point costs and the decreasing-cost order
    int32_t *d_order = nullptr;                 // [P]
    unsigned long long *d_cost = nullptr;       // [P] elimination steps per frequency
    unsigned long long *d_work_counter = nullptr;
    unsigned long long *d_exec = nullptr;   // executed formal-solve steps (profile mode)
    bool traced = false;
    int64_t *d_roff = nullptr;
    int32_t *d_rcells = nullptr;
    int64_t total_cells = 0;
    int64_t total_steps = 0;
    int max_len = 0;

    // work buffers (sized for P)
    void *d_lc = nullptr;  // line coefficients
    double *d_pops_a = nullptr, *d_pops_b = nullptr;
    double *d_J = nullptr, *d_Jeff = nullptr, *d_L = nullptr;
    uint8_t *d_flags = nullptr;
    nlte::ConvPartial *d_partials = nullptr;
    int64_t n_partials_cap = 0;
    nlte::ConvResult *d_conv = nullptr;
    nlte::ConvResult *h_conv = nullptr;  // pinned
    int32_t *d_active = nullptr;         // models still iterating
    int32_t *h_active = nullptr;         // pinned
    int64_t *d_maser = nullptr;

    // band ALO: outputs of the band formal solve and the coupled solve's work arrays
    int32_t *d_first = nullptr;          // [P][n_rays]
    bool first_valid = false;
    double *d_Jb = nullptr, *d_Ld = nullptr, *d_Ln = nullptr;
    double *d_bLU = nullptr, *d_bcpl = nullptr, *d_bx0 = nullptr;
    int32_t *d_bpiv = nullptr;
    double *d_bvec = nullptr;            // 8 vectors of [P][n_lev]
    double *d_bpart = nullptr, *d_bdot = nullptr, *h_bdot = nullptr;
    unsigned long long *d_bbad = nullptr, *h_bbad = nullptr;
    int64_t band_dims[5] = {0, 0, 0, 0, 0};   // P, n_lev, n_lines, n_rays, n_models the buffers were sized for
    uint8_t *d_bmodel_bad = nullptr;     // [n_models]
    std::vector<uint8_t> h_bmodel_bad;

    std::vector<double> dir_host;        // [n_rays][3] as set

    // scattering: opacity and the ALI's J_nu in two buffers (last one written: jnu_last)
    double *d_chi_sca = nullptr;         // [P][n_lines]
    double *d_chi_dip = nullptr;         // [P][n_lines][3]
    bool scat_on = false;
    bool dip_on = false;
    double *d_jnu[2] = {nullptr, nullptr};  // [P][n_lines][n_q] each
    int64_t jnu_elems = 0;
    int jnu_last = -1;
    bool q_ascending = false;
    bool q_uniform = false;          // evenly spaced offsets (spacing 1/q_inv_h)
    double q_inv_h = 0.0;

    // imaging: channel velocities
    double *d_vch = nullptr;
    int vch_cap = 0;

    // Ng acceleration: ring of the last M iterates and per-model work arrays
    double *d_ng_hist = nullptr;     // [M][P][n_lev]
    int64_t ng_hist_elems = 0;       // capacity in doubles
    double *d_ng_part = nullptr, *d_ng_coef = nullptr;
    uint8_t *d_ng_ok = nullptr;
    unsigned long long *d_ng_rej = nullptr;
    int ng_models_cap = 0;

    // launch choices and the captured ALI iterations (cur -> next, next -> cur)
    nlte::SolveConfig cfg;
    int n_cu = 0;
    std::string device_name;
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    const double *graph_buf[2] = {nullptr, nullptr};

    // warm-start network
    nlte::MlpState mlp;

    // profiling
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    nlte::KernelStat st_line_coef, st_formal, st_stateq, st_lte, st_trace;
    nlte::KernelStat st_features, st_mlp_forward, st_mlp_train, st_mlp_update, st_image;
};

namespace nlte {

// 1 if every point of this block (indices blockIdx.x * blockDim.x + [0, blockDim.x), cut
// at P) belongs to one model; models are contiguous index ranges, so the first and the
// last point decide.  0 for an empty block or without a point-to-model map.
__device__ inline int block_in_one_model(const int32_t *model_of, int64_t P)
{
    const int64_t p0 = blockIdx.x * (int64_t)blockDim.x;
    if (model_of == nullptr || p0 >= P) return 0;
    const int64_t p1 = (p0 + blockDim.x < P ? p0 + blockDim.x : P) - 1;
    return model_of[p0] == model_of[p1];
}

// Launchers (each enqueues on `stream`; return hipSuccess or the launch error).
hipError_t launch_setup_points(const double *pos, const double *vel, const double *nh2,
                               const double *T, const double *vturb, const double *X,
                               double mass, int64_t P, CellRec *cell, hipStream_t s);
hipError_t launch_lte(const SpeciesDev &sp, const CellRec *cell, const double *T, int64_t P,
                      double *pops, hipStream_t s);
// Neighbour slot of a point for the ray walk: the neighbour's position and index (m < 0:
// an unused slot), k slots per point back to back.
struct __align__(32) NbrEntry {
    double x, y, z;
    int32_t m, pad;
};
hipError_t launch_nbr_table(const CellRec *cell, const int32_t *nbr, int k, int64_t P, NbrEntry *tab,
                            hipStream_t s);
hipError_t launch_walk_count(const CellRec *cell, const NbrEntry *tab, int k, const uint8_t *bnd,
                             const double *dir, int n_rays, int64_t P, int64_t *len,
                             hipStream_t s);
hipError_t launch_walk_fill(const CellRec *cell, const NbrEntry *tab, int k, const uint8_t *bnd,
                            const double *dir, int n_rays, int64_t P, const int64_t *off,
                            int32_t *cells, hipStream_t s);
hipError_t scan_lengths(int64_t *len_then_off, int64_t n, void *tmp, size_t *tmp_bytes,
                        hipStream_t s);
hipError_t launch_line_coef(const SpeciesDev &sp, const CellRec *cell, const double *pops,
                            int64_t P, int fp32, void *lc, int64_t *maser_count, hipStream_t s);
hipError_t launch_formal_solve(const SolveArgs &a, const SolveConfig &cfg, int fp32, hipStream_t s);
hipError_t launch_formal_solve_f64(const SolveArgs &a, const SolveConfig &cfg, hipStream_t s);
hipError_t launch_formal_solve_f32(const SolveArgs &a, const SolveConfig &cfg, hipStream_t s);
// dynamic LDS bytes of one formal-solve workgroup with lpl lines per lane and ns staged nodes
size_t formal_solve_lds_f64(int lpl, int ns);
size_t formal_solve_lds_f32(int lpl, int ns);
// the formal-solve kernel's static LDS (its exponential table and work-queue slot, 136 bytes)
// rounded up, and the unit in which the hardware allocates a workgroup's LDS
constexpr size_t kFsStaticLds = 256;
constexpr size_t kLdsGranule = 512;
hipError_t launch_formal_solve_band(const SolveArgs &a, hipStream_t s);
hipError_t launch_count_steps(const SolveArgs &a, int64_t *steps, unsigned long long *point_cost,
                              hipStream_t s);
hipError_t sort_by_cost(unsigned long long *cost, int32_t *order, int64_t P, hipStream_t s);
hipError_t morton_order(const CellRec *cell, const int32_t *model_of, const double *box, const int64_t *off,
                        int n_models, int64_t P, int32_t *order, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s);
hipError_t launch_model_update(int n_models, unsigned long long *change, uint8_t *done, int32_t *iters,
                               double *last, double tol, int32_t *active, hipStream_t s);
hipError_t launch_stateq(const SpeciesDev &sp, const CellRec *cell, const double *nh2,
                         const double *T, int64_t P, int use_alo, const double *pops_old,
                         const double *J, const double *Jeff, const double *L, double *pops_new,
                         uint8_t *flags, ConvPartial *partials, int64_t n_blocks,
                         const uint8_t *model_done, const int32_t *model_of,
                         unsigned long long *model_change, hipStream_t s);
int64_t stateq_blocks(int64_t P);
hipError_t launch_conv_final(const ConvPartial *partials, int64_t n, ConvResult *out,
                             hipStream_t s);

// band ALO
hipError_t launch_first_cells(const int64_t *roff, const int32_t *rcells, int64_t n, int32_t *first, hipStream_t s);
hipError_t launch_band_setup(const BandArgs &b, const SpeciesDev &sp, const CellRec *cell, const double *nh2,
                             const double *T, const double *old, hipStream_t s);
hipError_t launch_band_apply(const BandArgs &b, const SpeciesDev &sp, const double *y, double *w, hipStream_t s);
int64_t band_dot_blocks(int64_t P);
hipError_t launch_band_dots(const DotArgs &d, const CellRec *cell, int n, int64_t P, double *part, double *out,
                            hipStream_t s);
hipError_t launch_band_lin(double *out, double a, const double *X, double b, const double *Y, double c,
                           const double *Z, int64_t N, hipStream_t s);
hipError_t launch_band_check_models(const double *x, int n, int64_t P, const int32_t *model_of, uint8_t *model_bad,
                                   hipStream_t s);
hipError_t launch_band_mask(const BandArgs &b, int n_lines, hipStream_t s);
hipError_t launch_band_finish(const double *x, const double *local, const uint8_t *model_bad, const double *old,
                              const CellRec *cell, int n, int64_t P, double *pops_new, uint8_t *flags,
                              ConvPartial *partials, const uint8_t *done, const int32_t *model_of,
                              unsigned long long *model_change, hipStream_t s);

// imaging
hipError_t launch_image(const ImageArgs &a, hipStream_t s);
hipError_t launch_image_plane(const CellRec *cell, double3 e1, double3 e2, int64_t P, double *xy, hipStream_t s);
hipError_t launch_formal_solve_scat(const ScatArgs &a, hipStream_t s);
hipError_t launch_jnu_start(const double *ibdy, int64_t P, int n_lines, int n_q, double *jnu, hipStream_t s);

// Ng acceleration
int ng_chunks();
hipError_t launch_ng(const NgHist &h, const CellRec *cell, const int64_t *off, const uint8_t *done,
                     const int32_t *model_of, int n_models, int n_lev, int64_t P, double *part, double *coef,
                     uint8_t *ok, double *out, unsigned long long *rejected, hipStream_t s);

// warm start
hipError_t launch_features(const CellRec *cell, const double *nh2, const double *T, const int32_t *nbr,
                           int k, const int64_t *roff, const int32_t *rcells, const double *dir, int R,
                           int64_t P, double *F, hipStream_t s);
int mlp_frag_count();
// training buffers of a batch: rows padded to 32 (ld), row chunks of the weight
// gradients, element counts of the layer inputs Ht (bfloat16) and output gradients DZt (FP32)
int mlp_train_ld(int batch);
int mlp_train_chunks(int batch);
size_t mlp_train_ht_count(int batch);
size_t mlp_train_dzt_count(int batch);
hipError_t launch_mlp_pack(const float *theta, const MlpDims &d, void *frags, hipStream_t s);
hipError_t launch_mlp_forward(const void *frags, const float *theta, const MlpDims &d, const float *X,
                              int64_t n, float *Y, hipStream_t s);
hipError_t launch_mlp_train(const void *frags, const float *theta, const MlpDims &d, const float *X, const float *T,
                            int64_t n, int64_t start, int batch, unsigned short *Ht, float *DZt, float *gpart,
                            float *lpart, hipStream_t s);
hipError_t launch_mlp_update(float *theta, float *m, float *v, void *frags, const MlpDims &d, const float *gpart,
                             int batch, int update, float lr, float b1, float b2, float eps, float c1, float c2,
                             const float *lpart, float inv_count, float *loss, float *grad_out, hipStream_t s);
hipError_t launch_mlp_standardise(const double *F, const MlpNorm &nm, int64_t P, float *X, hipStream_t s);
hipError_t launch_mlp_targets(const SpeciesDev &sp, const double *pops, const CellRec *cell, const double *T,
                              int64_t P, float *Tg, hipStream_t s);
hipError_t launch_mlp_populations(const SpeciesDev &sp, const float *Y, const CellRec *cell, const double *T,
                                  int64_t P, double *pops, unsigned long long *n_bad, hipStream_t s);

}  // namespace nlte
