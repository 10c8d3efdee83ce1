// Internal declarations of libfdlb (host structures, device argument blocks,
// kernel launchers).  Not part of the public ABI (include/fdlb.h is).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/fdlb.h"

namespace fdlb {

struct Error {
    int code;
    std::string msg;
    Error(int c, std::string m) : code(c), msg(std::move(m)) {}
};

void hip_check(hipError_t e, const char* what);
#define FDLB_HIP(call) ::fdlb::hip_check((call), #call)

void quad_half_range(int n, double* nodes, double* weights);
void quad_full_range(int n, double* nodes, double* weights);

enum { BOTTOM = 0, TOP = 1, LEFT = 2, RIGHT = 3 };

// Per-velocity constants, grouped by quadrant (sign of xi_x, sign of xi_y).
// ow* = omega * w-terms (relaxation), w* = w-terms (wall emission).
template <class T>
struct VelEntry {
    T ow, owx, owy;   // omega w, omega w xi_x, omega w xi_y
    T w, wx, wy;      // w, w xi_x, w xi_y
    T xx, xy;         // xi_x, xi_y
    T nux, nuy;       // dt |xi_x| N_x, dt |xi_y| N_y (0 along a periodic single-cell axis)
    int32_t alpha;    // plane index of this velocity in the state
    float pt;         // pseudo-time stretch of this velocity (steady iterations with local steps)
    // byte offset of that plane in a population buffer of type T (alpha * plane * sizeof(T)); held
    // at 4-byte alignment so that the float table keeps the alignment, and the compiler the load
    // grouping, that the bandwidth-bound tiles were tuned with
    int64_t off __attribute__((packed, aligned(4)));
};

// Per-wall constants of Eq. (9) in deviation form (double).  For the wall's
// inward normal n and tangent t, over the arriving half (xi . n < 0):
// A = sum |xi_n| w, Bn = sum |xi_n| w xi_n, Bt = sum |xi_n| w xi_t; k = 1 / E with
// E = sum xi_n w over the leaving half (the flux the emission carries per unit wall
// density; (2 pi)^(-1/2) for a half-range rule), so rho_w = k (A + arriving flux of h);
// c0 = k A - 1 (zero in exact arithmetic for the symmetric rules).
struct WallConst {
    double A, Bn, Bt, c0, k, u;
    int32_t active;
    int32_t pad;
};

// Everything the step kernel needs, passed by value.
template <class T>
struct StepArgs {
    const T* src;
    T* dst;
    const double* mom_in; // [3][ny][nx]: sum h, sum xi_x h, sum xi_y h of src (always double)
    double* mom_out;      // same for dst
    const double* phi_in; // [4][L]: sum over arriving half of |xi_n| h at each wall cell of src
    double* phi_out;
    double* partials;     // [nblocks][3]: sum |du|^2, sum |u|^2, max |u|^2 of this step
    const double* prev_partials;  // the previous step's, reduced here when prev_nb > 0
    double* ctrl;         // control block (freeze flags; block 0 records the previous step)
    const VelEntry<T>* vel;
    int32_t quad_begin[5];
    int32_t nx, ny, L;
    int32_t tiles_x, tiles_y;
    int32_t prev_nb;      // blocks of the previous step whose partials are still unreduced, or 0
    int32_t pseudo;       // 1: store h + pt (S h - h) instead of S h (selects the kernel variant)
    int64_t plane;        // nx * ny
    T omega;              // dt / Kn in the storage type
    T pad1;
    double omega_d;       // dt / Kn
    WallConst wall[4];
};

// A compiled tile shape of the step kernel.
struct TileShape {
    int vx;    // cells per lane along x (vector width)
    int lx;    // lanes along x in a wave (64 / lx lanes along y)
    int k;     // rows per lane
    int wpb;   // waves per block stacked along y
    int wa;    // waves per block sharing one tile, splitting the velocities
    int wx;    // waves per block side by side along x
    int nt;    // non-temporal population stores
    int pd;    // velocity planes whose loads are in flight beyond the current one
    int tile_w() const { return vx * lx * wx; }
    int tile_h() const { return (64 / lx) * k * wpb; }
};

// Batch launch: which problem and tile a block works on.
struct BlockMap {
    int32_t inst;   // problem index, -1 for a padding block
    int32_t local;  // block index within the problem
    int32_t nb;     // blocks of the problem
    int32_t pad;
};

// Batch reduction: one entry per problem.
struct ReduceArgs {
    const double* partials;
    double* ctrl;
    int32_t nb;          // <= 0: skip
    int32_t wave_order;  // 1: sum in the single-wave order of the inline reduction
};

// Velocity-local pseudo-time steps: the largest stretch of a velocity's step.
constexpr double FDLB_PSEUDO_MAX = 64.0;

// Residual partials of a launch with at most this many blocks are reduced inside the next step
// kernel (every wave of it sums them in the same order) instead of by a kernel of their own;
// one single-wave reduction closes every chunk of steps.
constexpr int INLINE_REDUCE_MAX_BLOCKS = 1024;

// When a FDLB_MIXED state leaves float during a steady solve: at a host check whose residual
// is below FDLB_MIXED_SWITCH_R, or once the lowest residual seen has not dropped by 10 % for
// FDLB_MIXED_STALL_STEPS steps (a float state stuck above the switch level).  Never when the
// tolerance is at or above the switch level: float reaches it alone.
struct MixedSwitch {
    bool on;
    double best = 1e300;
    int64_t best_step;
    MixedSwitch(bool enabled, double start_step) : on(enabled), best_step((int64_t)start_step) {}
    bool update(double residual, int64_t step);  // true: switch now
};

const std::vector<TileShape>& tile_shapes(int precision);
int heuristic_tile_for(int precision, int nx, int ny, bool periodic_x, bool periodic_y);
bool tile_fits(const TileShape& t, int nx, int ny, bool periodic_x, bool periodic_y);

// Launchers (kernels.hip).  All enqueue on `stream` and return immediately.
template <class T>
void launch_step(int tile, const StepArgs<T>& a, int nblocks, hipStream_t stream);
void launch_reduce(const double* partials, int nblocks, double* ctrl, int64_t inc, hipStream_t stream);
void launch_reduce_wave(const double* partials, int nblocks, double* ctrl, hipStream_t stream);
template <class T>
void launch_batch_step(int tile, const BlockMap* map, const StepArgs<T>* args, int nblocks, bool pseudo,
                       hipStream_t stream);
void launch_batch_reduce(const ReduceArgs* ra, int n, hipStream_t stream);
template <class T>
void launch_seed(T* h, int q, int64_t plane, const VelEntry<double>* vel, const double* rho,
                 const double* ux, const double* uy, const float* frho, const float* fux,
                 const float* fuy, const double* mass_scale, hipStream_t stream);
template <class T>
void launch_moments(const T* h, double* mom, double* phi, const VelEntry<T>* vel, int q, int nx, int ny,
                    int L, const WallConst* d_wall, hipStream_t stream);
template <class T>
void launch_post(const T* h, const VelEntry<double>* vel, int q, int nx, int ny, double omega,
                 double* out /* [4][ny][nx] */, hipStream_t stream);
template <class T>
void launch_wall_profile(const T* h, const VelEntry<double>* vel, int q, int nx, int ny, int wall,
                         const WallConst* host_wc, double omega, double* out /* [3][n] */,
                         hipStream_t stream);
// Planes [a0, a1) of the state <-> raw populations f = w + h in a compact double buffer.
template <class T>
void launch_to_raw(const T* h, const double* w_nat, int a0, int a1, int64_t plane, double* f,
                   hipStream_t stream);
template <class T>
void launch_from_raw(const double* f, const double* w_nat, int a0, int a1, int64_t plane, T* h,
                     hipStream_t stream);
void launch_mass_scale(const float* frho, int64_t cells, double* scale_out, hipStream_t stream);
void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t stream, int mode = FDLB_COPY_NT);
void launch_widen(const float* src, double* dst, int64_t n, hipStream_t stream);
// out[8 i + j] = ptrs[i][j], j < 8: the first control doubles of n problems in one array.
void launch_gather_ctrl(const double* const* ptrs, int n, double* out, hipStream_t stream);
// The first 8 doubles of a control block: step 0, nothing recorded, no freeze request.
void launch_ctrl_reset(double* ctrl, hipStream_t stream);
// On-disk cache of autotuned tiles (tunecache.cpp): enabled by a non-empty path.
void set_tune_cache_path(const char* path);
bool tune_cache_enabled();
std::string tune_key_prefix();  // device and compiled tile table
bool tune_cache_get(const std::string& key, int& tile, int& tile_alt, double& ms);
void tune_cache_put(const std::string& key, int tile, int tile_alt, double ms);

// Device address of the library's static workspace (FDLB_STATIC_SCRATCH_BYTES) on the current
// device, looked up on the first call per device (scratch.hip).
char* static_scratch();

// Warm-start network (mlp.hip / mlp.cpp).
constexpr int MLP_WIDTH = 128;     // hidden width (the matrix-core tiles assume it)
constexpr int MLP_TILE = 64;       // samples per block of the inference kernel
constexpr int MLP_TRAIN_TILE = 32; // samples per block of the training kernel
constexpr int MLP_SLICE = 256;     // samples per block of the hidden weight-gradient kernel
constexpr int MLP_MAX_HIDDEN = 8;  // hidden layers

struct MlpArgs {
    const float* params;        // flat: W_0, b_0, ..., W_L, b_L (W row-major by output)
    const uint16_t* wbf;        // bf16 hidden-to-hidden weights [hidden-1][128][128], [o][i]
    const uint16_t* wbfT;       // same, transposed, [i][o]
    const float* in;            // [.][3] encoded inputs (unless cells_nx > 0)
    const int32_t* rows;        // optional: sample g reads row rows[g] of in and target
    const float* target;        // [.][3]
    float* out;                 // [n][3] outputs (sample order, inference)
    uint16_t* hT;               // training: bf16 h_l, [hidden-1][n_cap/16][128][16] (l = 0..hidden-2)
    uint16_t* dzT;              // training: bf16 dE/dz_l, [hidden-1][n_cap/16][128][16] (l = 1..hidden-1)
    float* part_w;              // [slices][hidden-1][128][128] hidden weight gradients per sample slice
    float* part_thin;           // [thin][nb_cap] the other parameters' gradients per training block
    double* loss_part;          // [nb_cap] per-block squared errors
    float *f_rho, *f_ux, *f_uy; // field outputs: rho = 1 + u_w y0, u = u_w (y1, y2)
    int64_t n, n_cap, nb_cap;   // samples; samples per hT/dzT layer (multiple of MLP_SLICE); part_thin row length
    int32_t hidden, P;
    int32_t off_w[MLP_MAX_HIDDEN + 1], off_b[MLP_MAX_HIDDEN + 1];
    int32_t cells_nx, cells_ny; // > 0: inputs are the cells of this grid
    float kn_feat;              // encoded log10 Kn for cell inputs
    float u_w;
    float inv_3n;               // 1 / (3 n)
    int32_t pad;
};

// Parameters that are not hidden-to-hidden weights ("thin": W_0, b_0, the hidden biases,
// W_L, b_L), numbered W_0 (3 x 128), b_0, b_1 .. b_{hidden-1}, W_L (3 x 128), b_L.
__host__ __device__ inline int mlp_thin_count(int hidden) { return 4 * MLP_WIDTH + (hidden - 1) * MLP_WIDTH + 3 * MLP_WIDTH + 3; }

void launch_mlp_weights_bf16(const MlpArgs& a, uint16_t* wbf, uint16_t* wbfT, hipStream_t s);
void launch_mlp_forward(const MlpArgs& a, hipStream_t s);
void launch_mlp_train(const MlpArgs& a, hipStream_t s);
void launch_mlp_wgrad(const MlpArgs& a, hipStream_t s);
// One Adam step: parameters, moments, hyper-parameters with the bias corrections c1 = 1 / (1 -
// b1^t), c2 = 1 / (1 - b2^t), and the bf16 weight copies it refreshes.
struct AdamArgs {
    float *p, *m, *v;
    float lr, b1, b2, eps, c1, c2;
    uint16_t *wbf, *wbfT;
};
void launch_mlp_reduce(const MlpArgs& a, float* grad, double inv_3n, double* loss, const AdamArgs* adam,
                       hipStream_t s);
void launch_mlp_adam(const MlpArgs& a, const float* g, const AdamArgs& adam, hipStream_t s);
void launch_field_samples(const double* post, int nx, int ny, float kn_feat, double inv_uw, float* in, float* target,
                          hipStream_t s);
// Encoded Knudsen-number input of the network: (log10 Kn + 0.5) / 1.5 maps [0.01, 10] to [-1, 1].
inline float mlp_kn_feature(double kn) { return (float)((std::log10(kn) + 0.5) / 1.5); }

// Control block layout (doubles) written by the reduce kernel.
enum CtrlSlot {
    CTRL_STEP = 0,        // steps since init (stored as double, exact below 2^53)
    CTRL_LAST_R = 1,      // residual of the last reduced step
    CTRL_FIRST_BELOW = 2, // step count when R first fell below tol, -1 if never
    CTRL_DIVERGED = 3,    // step count of the first non-finite / runaway step, -1 if none
    CTRL_MAXU = 4,        // max |u| of the last step
    CTRL_TOL = 5,         // tolerance the reduce kernel compares against
    CTRL_FREEZE = 6,      // 1: stop updating once converged or diverged (steady solves)
    CTRL_HOST = 7,        // not used by the kernels
    CTRL_RING = 8,        // ring of residuals, CTRL_RING_LEN entries
};
constexpr int CTRL_RING_LEN = 4096;
constexpr int CTRL_DOUBLES = CTRL_RING + CTRL_RING_LEN;

}  // namespace fdlb

// ---- the opaque handles -------------------------------------------------------
struct fdlb_problem {
    fdlb_problem_desc d{};
    int q = 0;
    std::vector<double> xi_x, xi_y, w;     // velocity order of the ABI
    double dt = 0, omega = 0;
    std::vector<double> pt;                // pseudo-time stretch per velocity (ABI order)
    bool pseudo = false;                   // steps use velocity-local pseudo-time steps
    double nux_scale = 0, nuy_scale = 0;   // N along a bounded axis, 0 along a periodic single-cell one
    fdlb::WallConst wall[4]{};
    int32_t quad_begin[5]{};
    std::vector<int> quad_order;           // velocity index of each table entry (quadrant-grouped)
    std::vector<fdlb::VelEntry<float>> vel32;   // the device velocity tables, built once at creation
    std::vector<fdlb::VelEntry<double>> vel64;
    int L = 0;                             // max(nx, ny): stride of the per-wall arrays
    int64_t plane = 0;                     // nx * ny
    int prec = FDLB_FP64;                  // precision the kernels run in now (FDLB_FP32 / FDLB_FP64)
    size_t elem = 0;                       // bytes per population in that precision (4 or 8)
    // layout (byte offsets into the state / workspace)
    size_t pop_bytes = 0, state_bytes = 0, work_bytes = 0;
    size_t off_mom = 0, mom_bytes = 0, off_phi = 0, phi_bytes = 0, off_part = 0, off_ctrl = 0,
           off_vel = 0, off_vel64 = 0, off_wall = 0, off_wnat = 0, off_io = 0, io_bytes = 0;
    int max_blocks = 0;
    int tile = -1;                         // tile shape in use (a shape of tile_shapes(prec))
    int tile_alt = -1;                     // FDLB_MIXED: the shape kept for the other precision
    // binding
    char* d_state = nullptr;
    char* d_work = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    bool seeded = false;
    int parity = 0;                        // population buffer holding the current state
    double* pinned = nullptr;              // small pinned host buffer for control reads (64 doubles)
    bool own_pinned = true;                // false: a slice of its batch's block, freed by the batch
    bool freeze_on = false;                // the device control block has the freeze flag set
    // captured graphs keyed by (steps per replay, precision, tile, starting parity)
    std::map<std::tuple<int, int, int, int>, hipGraphExec_t> graphs;
    ~fdlb_problem();
};

// ---- hybrid half-range / full-range channel (hybrid.hip, hybrid.cpp) ---------------------
namespace fdlb {

// One channel of a hybrid batch as the kernels see it.  Its table (doubles, at tab_off) holds
// x nodes, x weights, layer y nodes, layer y weights, layer Courant numbers, bulk y nodes, bulk
// y weights, bulk Courant numbers, the layer->bulk map [nf][nh] and the bulk->layer map
// [nh][nf], in that order.
struct HybChan {
    int32_t ny, layer, nx, nh, nf, qh, qf, active;  // nh, nf: y nodes of the layer / bulk sets
    int64_t state_off;   // doubles into the state arena
    int64_t tab_off;     // doubles into the table
    int64_t hist_off;    // doubles into the residual ring
    int32_t ntab, pad;
    double omega;        // dt / Kn
    double e_inv;        // 1 / sum_{xi_y > 0} xi_y w over the layer set (wall density per arriving flux)
    double u_bottom, u_top;
    // per plate (0 bottom, 1 top), sums over its arriving half of the layer set:
    // A = sum |xi_y| w, Bx = sum |xi_y| xi_x w, By = sum |xi_y| xi_y w (the arriving flux of an
    // equilibrium w (rho + xi . j) is rho A + j_x Bx + j_y By)
    double wA[2], wBx[2], wBy[2];
};

// Per-channel control block, written by the march kernel.
struct HybCtl {
    int64_t steps;        // steps taken since seeding
    int64_t first_below;  // step count at which the residual first fell below tol, or -1
    double residual;      // residual of the last step
    int32_t status;       // 0 marching, 1 converged, 2 non-finite residual
    int32_t pad;
};

constexpr int HYB_THREADS = 256;         // seeding and output kernels
constexpr int HYB_MARCH_THREADS = 512;   // the march kernel: eight waves
constexpr int HYB_RING = 1024;   // residuals kept per channel (the most recent ones)

// Plane groups per chunk of 64 cells in the march kernel: enough work items for every wave of
// the block when the channel has few chunks.
__host__ __device__ inline int hyb_groups(int chunks) {
    const int g = (HYB_MARCH_THREADS / 64) / (chunks > 0 ? chunks : 1);
    return g > 1 ? g : 1;
}

// LDS bytes a channel's march needs.
size_t hybrid_lds_bytes(const HybChan& c);

// Launchers (hybrid.hip); asynchronous on `stream`.
void launch_hybrid_march(const HybChan* d_chans, int n, const double* d_tab, double* d_state, HybCtl* d_ctl,
                         double* d_ring, int64_t nsteps, double tol, int solve, size_t lds, hipStream_t stream);
void launch_hybrid_seed(const HybChan* d_chans, int ch, int ny, const double* d_tab, double* d_state,
                        const double* d_fields, hipStream_t stream);
void launch_hybrid_post(const HybChan* d_chans, int ch, const double* d_tab, const double* d_state,
                        double* d_out, size_t lds, hipStream_t stream);
void hybrid_allow_lds(size_t bytes);

}  // namespace fdlb
