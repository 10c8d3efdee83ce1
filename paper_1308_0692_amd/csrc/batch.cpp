// Batched steady solves: many independent problems (different Kn, grids and velocity sets,
// one precision) advanced together, one step-kernel launch per time step for all of them.
// Each problem's residual is reduced as for a single problem: by an extra block of the next
// launch (small problems, closed by one reduction launch per chunk) or by a shared reduction
// launch after every step (large problems).  In FDLB_MIXED each problem leaves float on its
// own; the batch then launches the float members and the double members as two groups.
//
// Every problem keeps its own state, workspace and control block inside two caller-owned
// arenas.  A block map assigns each block of the launch to (problem, tile); each problem's
// blocks start at a multiple of 8 so that the XCD-aware tile order holds per problem.  A
// problem whose residual falls below the tolerance (or diverges) freezes on the device at
// that step; the host drops it from the block map at the next check, so the remaining
// problems keep the chip.  Chunks of `check_every` steps are replayed as captured graphs.
#include <algorithm>
#include <cstdio>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>
#include <type_traits>

#include "fdlb_internal.h"

namespace fdlb {
void promote(fdlb_problem& p);
void promote_async(fdlb_problem& p);
void init_rest_async(fdlb_problem& p);
double* partials_of(fdlb_problem& p, int parity);
void field_samples(fdlb_problem& p, float* in, float* target);
void build_problem(fdlb_problem& p, const fdlb_problem_desc& d);
void bind(fdlb_problem& p, void* d_state, void* d_work, void* stream);
void init_equilibrium(fdlb_problem& p, const double* rho, const double* ux, const double* uy, int renorm);
void init_equilibrium_dev(fdlb_problem& p, const float* rho, const float* ux, const float* uy, int renorm);
void moments(fdlb_problem& p, double* rho, double* ux, double* uy, double* pxy);
void wall_profile(fdlb_problem& p, int wall, double* rho, double* ut, double* pxy);
void state_download(fdlb_problem& p, double* f);
void state_upload(fdlb_problem& p, const double* f);
}  // namespace fdlb

// The members that run in one precision: their block map and step arguments.
struct BatchGroup {
    bool used = false;
    int tile = -1;            // a shape of tile_shapes(prec)
    size_t off_map = 0;       // BlockMap[max_map]
    size_t off_args = 0;      // StepArgs<T>[2 parities][2 (reduces its predecessor)][n]
    int max_map = 0;
    int map_blocks = 0;
};

struct fdlb_batch {
    std::vector<std::unique_ptr<fdlb_problem>> probs;
    int precision = FDLB_FP32;
    BatchGroup grp[2];              // [0]: float kernels, [1]: double kernels
    std::vector<size_t> state_off, work_off;
    size_t state_bytes = 0, work_bytes = 0;
    size_t off_rargs = 0;           // ReduceArgs[2 parities][2: per step, end of chunk][n]
    bool step_reduce = false;       // some member reduces every step with a kernel of its own
    bool end_reduce = false;        // some member reduces inline (closed at the end of a chunk)
    size_t off_ctrlptr = 0, off_ctrlbuf = 0;
    int retile_members = 8;         // re-choose tiles once at most this many instances remain (0: never)
    bool pseudo = false;            // every member steps with velocity-local pseudo-time steps
    char* d_state = nullptr;
    char* d_work = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    double* pinned = nullptr;       // n x 8 control doubles
    double* member_pinned = nullptr;  // n x 64 doubles: the members' staging buffers, one allocation
    std::vector<int> active;        // problems in the current block maps
    int map_version = 0;
    // (k, parity, map version, float tile, double tile)
    std::map<std::tuple<int, int, int, int, int>, hipGraphExec_t> graphs;
    ~fdlb_batch() {
        for (auto& kv : graphs) (void)hipGraphExecDestroy(kv.second);
        if (pinned) (void)hipHostFree(pinned);
        probs.clear();  // the members first: their staging buffers are slices of member_pinned
        if (member_pinned) (void)hipHostFree(member_pinned);
    }
};

namespace fdlb {

namespace {
size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

int nblocks_tile(const fdlb_problem& p, const TileShape& t) {
    return ((p.d.nx + t.tile_w() - 1) / t.tile_w()) * ((p.d.ny + t.tile_h() - 1) / t.tile_h());
}

int prec_of_group(int g) { return g == 0 ? FDLB_FP32 : FDLB_FP64; }
int group_of(const fdlb_problem& p) { return p.prec == FDLB_FP32 ? 0 : 1; }
// The group the public tile calls act on: float unless the batch is all double.
int primary_group(const fdlb_batch& b) { return b.precision == FDLB_FP64 ? 1 : 0; }

bool tile_fits_all(const fdlb_batch& b, int g, int tile) {
    const TileShape& t = tile_shapes(prec_of_group(g))[tile];
    for (auto& p : b.probs) {
        if (!tile_fits(t, p->d.nx, p->d.ny, p->d.periodic_x, p->d.periodic_y)) return false;
        if (nblocks_tile(*p, t) > p->max_blocks) return false;
    }
    return true;
}

int member_blocks(const fdlb_batch& b, const fdlb_problem& p) {
    const int g = group_of(p);
    return nblocks_tile(p, tile_shapes(prec_of_group(g))[b.grp[g].tile]);
}

double* ctrl_of(fdlb_problem& p) { return (double*)(p.d_work + p.off_ctrl); }
}  // namespace

static void group_set_tile(fdlb_batch& b, int g, int tile);

void batch_create(fdlb_batch& b, const fdlb_problem_desc* descs, int n) {
    if (!descs || n < 1) throw Error(FDLB_EINVAL, "a batch needs at least one problem");
    b.precision = descs[0].precision;
    for (int i = 0; i < n; ++i) {
        if (descs[i].precision != b.precision) throw Error(FDLB_EINVAL, "all problems of a batch share the precision");
        auto p = std::make_unique<fdlb_problem>();
        try {
            build_problem(*p, descs[i]);
        } catch (const Error& e) {
            throw Error(e.code, "problem " + std::to_string(i) + ": " + e.msg);
        }
        b.probs.push_back(std::move(p));
    }
    // Arenas: each problem's state and workspace, then the batch region.
    size_t so = 0, wo = 0;
    for (auto& p : b.probs) {
        b.state_off.push_back(so);
        b.work_off.push_back(wo);
        so += align256(p->state_bytes);
        wo += align256(p->work_bytes);
    }
    b.grp[0].used = b.precision != FDLB_FP64;
    b.grp[1].used = b.precision != FDLB_FP32;
    for (int g = 0; g < 2; ++g) {
        BatchGroup& G = b.grp[g];
        if (!G.used) continue;
        int maxmap = 0;
        for (const TileShape& t : tile_shapes(prec_of_group(g))) {
            int tot = 0;
            for (auto& p : b.probs) tot += (nblocks_tile(*p, t) + 1 + 7) / 8 * 8;  // + reduction block
            maxmap = std::max(maxmap, tot);
        }
        G.max_map = maxmap;
        G.off_map = wo;
        wo += align256((size_t)maxmap * sizeof(BlockMap));
        G.off_args = wo;
        wo += align256(4 * (size_t)n * (g == 0 ? sizeof(StepArgs<float>) : sizeof(StepArgs<double>)));
    }
    b.off_rargs = wo;
    wo += align256(4 * (size_t)n * sizeof(ReduceArgs));
    b.off_ctrlptr = wo;  // every member's control block, gathered for one host read per check
    wo += align256((size_t)n * sizeof(double*));
    b.off_ctrlbuf = wo;
    wo += align256((size_t)n * 8 * sizeof(double));
    b.state_bytes = so;
    b.work_bytes = wo;
    // Default tiles: the built-in choice for the largest problem if it fits all, else any that does.
    int big = 0;
    for (int i = 1; i < n; ++i)
        if (b.probs[i]->plane * b.probs[i]->q > b.probs[big]->plane * b.probs[big]->q) big = i;
    const fdlb_problem& pb = *b.probs[big];
    for (int g = 0; g < 2; ++g) {
        if (!b.grp[g].used) continue;
        const int prec = prec_of_group(g);
        int t = heuristic_tile_for(prec, pb.d.nx, pb.d.ny, pb.d.periodic_x, pb.d.periodic_y);
        if (!tile_fits_all(b, g, t)) {
            t = -1;
            for (int i = 0; i < (int)tile_shapes(prec).size(); ++i)
                if (tile_fits_all(b, g, i)) {
                    t = i;
                    break;
                }
            if (t < 0) throw Error(FDLB_EINVAL, "no compiled tile shape fits every problem of the batch");
        }
        group_set_tile(b, g, t);
    }
}

// Each member keeps the group tiles in its own handle (tile: active precision, tile_alt:
// the other one), so that its solo calls agree with the batch.
static void group_set_tile(fdlb_batch& b, int g, int tile) {
    const int prec = prec_of_group(g);
    if (tile < 0 || tile >= (int)tile_shapes(prec).size()) throw Error(FDLB_EINVAL, "tile index out of range");
    if (!tile_fits_all(b, g, tile)) throw Error(FDLB_EINVAL, "tile shape does not fit every problem of the batch");
    b.grp[g].tile = tile;
    for (auto& p : b.probs) {
        if (p->prec == prec) p->tile = tile;
        else p->tile_alt = tile;
    }
}

void batch_set_tile(fdlb_batch& b, int tile) { group_set_tile(b, primary_group(b), tile); }

void batch_bind(fdlb_batch& b, void* d_state, void* d_work, void* stream) {
    if (!d_state || !d_work) throw Error(FDLB_EINVAL, "device buffers must not be NULL");
    for (auto& kv : b.graphs) (void)hipGraphExecDestroy(kv.second);
    b.graphs.clear();
    b.d_state = (char*)d_state;
    b.d_work = (char*)d_work;
    b.stream = (hipStream_t)stream;
    // One pinned allocation for all members' staging buffers (thousands of small pinned
    // allocations, and their frees, cost about a millisecond each).
    if (!b.member_pinned) {
        FDLB_HIP(hipHostMalloc((void**)&b.member_pinned, b.probs.size() * 64 * sizeof(double), hipHostMallocDefault));
        for (size_t i = 0; i < b.probs.size(); ++i) {
            b.probs[i]->pinned = b.member_pinned + 64 * i;
            b.probs[i]->own_pinned = false;
        }
    }
    for (size_t i = 0; i < b.probs.size(); ++i) bind(*b.probs[i], b.d_state + b.state_off[i], b.d_work + b.work_off[i], stream);
    if (!b.pinned)
        FDLB_HIP(hipHostMalloc((void**)&b.pinned, b.probs.size() * 8 * sizeof(double), hipHostMallocDefault));
    {
        std::vector<const double*> ptrs;
        for (auto& p : b.probs) ptrs.push_back(ctrl_of(*p));
        FDLB_HIP(hipMemcpyAsync(b.d_work + b.off_ctrlptr, ptrs.data(), ptrs.size() * sizeof(ptrs[0]),
                                hipMemcpyHostToDevice, b.stream));
        FDLB_HIP(hipStreamSynchronize(b.stream));  // ptrs is a host temporary
    }
    b.bound = true;
}

static fdlb_problem& inst(fdlb_batch& b, int i) {
    if (i < 0 || i >= (int)b.probs.size()) throw Error(FDLB_EINVAL, "instance index out of range");
    return *b.probs[i];
}

void batch_init_equilibrium(fdlb_batch& b, int i, const double* rho, const double* ux, const double* uy, int renorm) {
    init_equilibrium(inst(b, i), rho, ux, uy, renorm);
}
void batch_init_equilibrium_dev(fdlb_batch& b, int i, const float* rho, const float* ux, const float* uy, int renorm) {
    init_equilibrium_dev(inst(b, i), rho, ux, uy, renorm);
}
void batch_moments(fdlb_batch& b, int i, double* rho, double* ux, double* uy, double* pxy) {
    moments(inst(b, i), rho, ux, uy, pxy);
}
void batch_wall_profile(fdlb_batch& b, int i, int wall, double* rho, double* ut, double* pxy) {
    wall_profile(inst(b, i), wall, rho, ut, pxy);
}
void batch_state_download(fdlb_batch& b, int i, double* f) { state_download(inst(b, i), f); }
void batch_state_upload(fdlb_batch& b, int i, const double* f) { state_upload(inst(b, i), f); }

template <class T>
static StepArgs<T> batch_step_args(fdlb_problem& p, int parity, int tile, bool prev) {
    constexpr bool f32 = std::is_same<T, float>::value;
    const TileShape& t = tile_shapes(f32 ? FDLB_FP32 : FDLB_FP64)[tile];
    const int nb = nblocks_tile(p, t);
    StepArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    char* pop = p.d_state;
    char* mom = p.d_work + p.off_mom;
    char* phi = p.d_work + p.off_phi;
    a.src = (const T*)(pop + (size_t)parity * p.pop_bytes);
    a.dst = (T*)(pop + (size_t)(parity ^ 1) * p.pop_bytes);
    a.mom_in = (const double*)(mom + (size_t)parity * p.mom_bytes);
    a.mom_out = (double*)(mom + (size_t)(parity ^ 1) * p.mom_bytes);
    a.phi_in = (const double*)(phi + (size_t)parity * p.phi_bytes);
    a.phi_out = (double*)(phi + (size_t)(parity ^ 1) * p.phi_bytes);
    a.partials = partials_of(p, parity);
    a.prev_partials = partials_of(p, parity ^ 1);
    a.prev_nb = prev && nb <= INLINE_REDUCE_MAX_BLOCKS ? nb : 0;
    a.pseudo = p.pseudo ? 1 : 0;
    a.ctrl = ctrl_of(p);
    a.vel = (const VelEntry<T>*)(p.d_work + (f32 ? p.off_vel : p.off_vel64));
    for (int i = 0; i < 5; ++i) a.quad_begin[i] = p.quad_begin[i];
    a.nx = p.d.nx;
    a.ny = p.d.ny;
    a.L = p.L;
    a.tiles_x = (p.d.nx + t.tile_w() - 1) / t.tile_w();
    a.tiles_y = (p.d.ny + t.tile_h() - 1) / t.tile_h();
    a.plane = p.plane;
    a.omega = (T)p.omega;
    a.omega_d = p.omega;
    for (int i = 0; i < 4; ++i) a.wall[i] = p.wall[i];
    return a;
}

// Reduce arguments, by the parity of the step's source buffer: a member with few blocks is
// reduced inline and closed at the end of a chunk (single-wave order), the others after every
// step; each member's partials are laid out by its group's tile.
static void upload_rargs(fdlb_batch& b) {
    const int n = (int)b.probs.size();
    std::vector<ReduceArgs> ra(4 * (size_t)n);
    b.step_reduce = b.end_reduce = false;
    for (int par = 0; par < 2; ++par)
        for (int kind = 0; kind < 2; ++kind)
            for (int i = 0; i < n; ++i) {
                fdlb_problem& p = *b.probs[i];
                const int nb = member_blocks(b, p);
                const bool inl = nb <= INLINE_REDUCE_MAX_BLOCKS;
                ReduceArgs& r = ra[(size_t)(par * 2 + kind) * n + i];
                r.partials = partials_of(p, par);
                r.ctrl = ctrl_of(p);
                r.nb = (kind == 1) == inl ? nb : 0;
                r.wave_order = kind;
                (inl ? b.end_reduce : b.step_reduce) = true;
            }
    FDLB_HIP(hipMemcpyAsync(b.d_work + b.off_rargs, ra.data(), ra.size() * sizeof(ReduceArgs), hipMemcpyHostToDevice,
                            b.stream));
    FDLB_HIP(hipStreamSynchronize(b.stream));
}

template <class T>
static void upload_group_args(fdlb_batch& b, int g) {
    const int n = (int)b.probs.size();
    std::vector<StepArgs<T>> a(4 * (size_t)n);
    for (int par = 0; par < 2; ++par)
        for (int prev = 0; prev < 2; ++prev)
            for (int i = 0; i < n; ++i)
                a[(size_t)(par * 2 + prev) * n + i] = batch_step_args<T>(*b.probs[i], par, b.grp[g].tile, prev != 0);
    FDLB_HIP(hipMemcpyAsync(b.d_work + b.grp[g].off_args, a.data(), a.size() * sizeof(a[0]), hipMemcpyHostToDevice,
                            b.stream));
    FDLB_HIP(hipStreamSynchronize(b.stream));  // a is a host temporary
}

// Upload the per-problem step arguments of every group (all members, both parities) and the
// reduce arguments.
static void upload_args(fdlb_batch& b) {
    if (b.grp[0].used) upload_group_args<float>(b, 0);
    if (b.grp[1].used) upload_group_args<double>(b, 1);
    upload_rargs(b);
}

// Block maps of the active problems, one per group.
static void upload_map(fdlb_batch& b) {
    for (int g = 0; g < 2; ++g) {
        BatchGroup& G = b.grp[g];
        if (!G.used) continue;
        std::vector<BlockMap> m;
        const TileShape& t = tile_shapes(prec_of_group(g))[G.tile];
        // Longest blocks first (more velocities per cell, then more blocks): the hardware hands
        // out blocks in index order, so the last ones to start are the short ones and the launch
        // ends with less of the chip idle.  A block's work depends only on (inst, local), so the
        // order changes no result.
        std::vector<int> order(b.active.begin(), b.active.end());
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            const fdlb_problem &px = *b.probs[x], &py = *b.probs[y];
            if (px.q != py.q) return px.q > py.q;
            return nblocks_tile(px, t) > nblocks_tile(py, t);
        });
        for (int i : order) {
            if (group_of(*b.probs[i]) != g) continue;
            const int nb = nblocks_tile(*b.probs[i], t);
            for (int l = 0; l < nb; ++l) m.push_back(BlockMap{i, l, nb, 0});
            // a problem reduced inline gets its reduction block (local == nb)
            if (nb <= INLINE_REDUCE_MAX_BLOCKS) m.push_back(BlockMap{i, nb, nb, 0});
            while (m.size() % 8) m.push_back(BlockMap{-1, 0, 0, 0});
        }
        G.map_blocks = (int)m.size();
        if (G.map_blocks > G.max_map) throw Error(FDLB_EINVAL, "block map overflow");
        if (!m.empty())
            FDLB_HIP(hipMemcpyAsync(b.d_work + G.off_map, m.data(), m.size() * sizeof(BlockMap), hipMemcpyHostToDevice,
                                    b.stream));
        FDLB_HIP(hipStreamSynchronize(b.stream));
    }
    ++b.map_version;
}

// One batch step from source parity `parity`; prev: the members that reduce inline reduce
// their previous step in this launch.
static void enqueue_batch_step(fdlb_batch& b, int parity, bool prev) {
    const int n = (int)b.probs.size();
    const size_t v = (size_t)(parity * 2 + (prev ? 1 : 0)) * n;
    for (int g = 0; g < 2; ++g) {
        const BatchGroup& G = b.grp[g];
        if (!G.used || G.map_blocks == 0) continue;
        const BlockMap* map = (const BlockMap*)(b.d_work + G.off_map);
        if (g == 0)
            launch_batch_step<float>(G.tile, map, (const StepArgs<float>*)(b.d_work + G.off_args) + v, G.map_blocks,
                                     b.pseudo, b.stream);
        else
            launch_batch_step<double>(G.tile, map, (const StepArgs<double>*)(b.d_work + G.off_args) + v,
                                      G.map_blocks, b.pseudo, b.stream);
    }
    if (b.step_reduce)
        launch_batch_reduce((const ReduceArgs*)(b.d_work + b.off_rargs) + (size_t)(parity * 2) * n, n, b.stream);
}

static void enqueue_batch_steps(fdlb_batch& b, int k, int parity) {
    const int n = (int)b.probs.size();
    for (int i = 0; i < k; ++i) enqueue_batch_step(b, parity ^ (i & 1), i > 0);
    if (k > 0 && b.end_reduce) {
        const int last = parity ^ ((k - 1) & 1);
        launch_batch_reduce((const ReduceArgs*)(b.d_work + b.off_rargs) + (size_t)(last * 2 + 1) * n, n, b.stream);
    }
}

static void enqueue_batch_chunk(fdlb_batch& b, int k, int parity, bool graph) {
    if (!graph) {
        enqueue_batch_steps(b, k, parity);
        return;
    }
    auto key = std::make_tuple(k, parity, b.map_version, b.grp[0].tile, b.grp[1].tile);
    auto it = b.graphs.find(key);
    if (it == b.graphs.end()) {
        // Graphs of an older block map are stale: drop them.
        for (auto g = b.graphs.begin(); g != b.graphs.end();) {
            if (std::get<2>(g->first) != b.map_version) {
                (void)hipGraphExecDestroy(g->second);
                g = b.graphs.erase(g);
            } else {
                ++g;
            }
        }
        hipGraph_t g;
        FDLB_HIP(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal));
        try {
            enqueue_batch_steps(b, k, parity);
        } catch (...) {
            hipGraph_t dummy;
            (void)hipStreamEndCapture(b.stream, &dummy);
            throw;
        }
        FDLB_HIP(hipStreamEndCapture(b.stream, &g));
        hipGraphExec_t ge;
        FDLB_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
        FDLB_HIP(hipGraphDestroy(g));
        it = b.graphs.emplace(key, ge).first;
    }
    FDLB_HIP(hipGraphLaunch(it->second, b.stream));
}

static void read_all_ctrl(fdlb_batch& b) {
    const int n = (int)b.probs.size();
    launch_gather_ctrl((const double* const*)(b.d_work + b.off_ctrlptr), n, (double*)(b.d_work + b.off_ctrlbuf),
                       b.stream);
    FDLB_HIP(hipMemcpyAsync(b.pinned, b.d_work + b.off_ctrlbuf, (size_t)n * 8 * sizeof(double),
                            hipMemcpyDeviceToHost, b.stream));
    FDLB_HIP(hipStreamSynchronize(b.stream));
}

int batch_solve(fdlb_batch& b, double tol, int64_t max_steps, int32_t check_every, int32_t use_graph,
                fdlb_report* reps) {
    if (!b.bound) throw Error(FDLB_ESTATE, "batch is not bound to device memory");
    if (!(tol >= 0) || max_steps < 0 || check_every < 1) throw Error(FDLB_EINVAL, "bad solve arguments");
    const int n = (int)b.probs.size();
    for (auto& p : b.probs)
        if (!p->seeded) throw Error(FDLB_ESTATE, "every problem of the batch must be initialised");
    read_all_ctrl(b);
    // All problems advance together, so they must share the buffer parity.
    const int parity0 = (int)((int64_t)b.pinned[CTRL_STEP] & 1);
    std::vector<double> base(n);
    for (int i = 0; i < n; ++i) {
        base[i] = b.pinned[8 * i + CTRL_STEP];
        if ((int)((int64_t)base[i] & 1) != parity0)
            throw Error(FDLB_ESTATE, "problems of a batch must have taken step counts of equal parity");
        double* h = b.pinned + 8 * i;
        h[CTRL_FIRST_BELOW] = -1.0;
        h[CTRL_DIVERGED] = -1.0;
        h[CTRL_TOL] = tol;
        h[CTRL_FREEZE] = 1.0;
        FDLB_HIP(hipMemcpyAsync(ctrl_of(*b.probs[i]) + CTRL_FIRST_BELOW, h + CTRL_FIRST_BELOW, 5 * sizeof(double),
                                hipMemcpyHostToDevice, b.stream));
        b.probs[i]->freeze_on = true;
    }
    FDLB_HIP(hipStreamSynchronize(b.stream));
    upload_args(b);
    b.active.clear();
    for (int i = 0; i < n; ++i) b.active.push_back(i);
    upload_map(b);
    const bool graph = use_graph && b.stream != nullptr && check_every >= 2;
    // The tail: once few instances remain, the launch is latency-bound and the shape chosen for
    // the full batch (many waves per tile, throughput) loses to the single-problem choice.
    const int saved_tile[2] = {b.grp[0].tile, b.grp[1].tile};
    bool may_retile = b.retile_members > 0 && n > b.retile_members;
    std::vector<int32_t> hlen(n, 0);
    std::vector<MixedSwitch> sw;
    std::vector<double> fp32_until(n);  // step count where a member's float phase ended, -1: not yet
    for (int i = 0; i < n; ++i) {
        const fdlb_problem& p = *b.probs[i];
        sw.emplace_back(p.d.precision == FDLB_MIXED && p.prec == FDLB_FP32 && tol < FDLB_MIXED_SWITCH_R, base[i]);
        fp32_until[i] = p.prec == FDLB_FP32 ? -1.0 : base[i];
    }
    const auto t0 = std::chrono::steady_clock::now();
    int64_t launched = 0;
    int parity = parity0;
    while (launched < max_steps && !b.active.empty()) {
        const int64_t k = std::min<int64_t>(check_every, max_steps - launched);
        enqueue_batch_chunk(b, (int)k, parity, graph && k == check_every);
        if (k & 1) parity ^= 1;
        launched += k;
        read_all_ctrl(b);
        std::vector<int> still;
        bool switched = false;
        for (int i : b.active) {
            const double* c = b.pinned + 8 * i;
            if (reps && reps[i].history && hlen[i] < reps[i].history_cap) reps[i].history[hlen[i]++] = c[CTRL_LAST_R];
            if (c[CTRL_FIRST_BELOW] >= 0 || c[CTRL_DIVERGED] >= 0) continue;
            still.push_back(i);
            fdlb_problem& p = *b.probs[i];
            if (p.prec == FDLB_FP32 && sw[i].update(c[CTRL_LAST_R], (int64_t)c[CTRL_STEP])) {
                p.parity = parity;  // every active member is at the batch's parity
                promote(p);
                fp32_until[i] = c[CTRL_STEP];
                switched = true;
            }
        }
        if (switched) upload_rargs(b);
        if (switched || still.size() != b.active.size()) {
            b.active = still;
            if (may_retile && !still.empty() && (int)still.size() <= b.retile_members) {
                may_retile = false;
                bool changed = false;
                for (int g = 0; g < 2; ++g) {
                    if (!b.grp[g].used) continue;
                    int big = -1;
                    for (int i : still)
                        if (group_of(*b.probs[i]) == g &&
                            (big < 0 || b.probs[i]->plane * b.probs[i]->q > b.probs[big]->plane * b.probs[big]->q))
                            big = i;
                    if (big < 0) continue;
                    const fdlb_problem& pb = *b.probs[big];
                    const int t = heuristic_tile_for(prec_of_group(g), pb.d.nx, pb.d.ny, pb.d.periodic_x, pb.d.periodic_y);
                    if (t != b.grp[g].tile && tile_fits_all(b, g, t)) {
                        group_set_tile(b, g, t);
                        changed = true;
                    }
                }
                if (changed) upload_args(b);
            }
            upload_map(b);
        }
    }
    for (int g = 0; g < 2; ++g)
        if (b.grp[g].used && b.grp[g].tile != saved_tile[g]) group_set_tile(b, g, saved_tile[g]);
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int status = FDLB_OK;
    for (int i = 0; i < n; ++i) {
        fdlb_problem& p = *b.probs[i];
        const double* c = b.pinned + 8 * i;
        int st = FDLB_ENOTCONVERGED;
        if (c[CTRL_DIVERGED] >= 0) st = FDLB_EDIVERGED;
        else if (c[CTRL_FIRST_BELOW] >= 0) st = FDLB_OK;
        if (st == FDLB_EDIVERGED) status = FDLB_EDIVERGED;
        else if (st == FDLB_ENOTCONVERGED && status == FDLB_OK) status = FDLB_ENOTCONVERGED;
        p.parity = (int)((int64_t)c[CTRL_STEP] & 1);
        if (reps) {
            fdlb_report& r = reps[i];
            r.steps = (int64_t)(c[CTRL_STEP] - base[i]);
            r.first_below = st == FDLB_OK ? (int64_t)(c[CTRL_FIRST_BELOW] - base[i]) : -1;
            r.residual = c[CTRL_LAST_R];
            r.wall_s = wall;
            const double upd = (double)r.steps * (double)p.plane * p.q;
            r.updates_per_s = wall > 0 ? upd / wall : 0;
            r.steps_fp32 = fp32_until[i] < 0 ? r.steps : (int64_t)(fp32_until[i] - base[i]);
            const double cell_q = (double)p.plane * p.q;
            r.bytes_per_s =
                wall > 0 ? cell_q * (8.0 * (double)r.steps_fp32 + 16.0 * (double)(r.steps - r.steps_fp32)) / wall : 0;
            r.status = st;
            r.history_len = hlen[i];
        }
    }
    return status;
}

// Time of one step of the whole batch on its current tiles: one untimed step (a shape's first
// launch also loads its code), one timed step, and, unless that step already took over twice the
// best time so far (its further steps would not change the choice), `steps` more timed steps.  A
// large batch's poor shapes thus cost two steps each instead of all of them.  `parity` follows
// the steps enqueued.
static double time_batch_shape(fdlb_batch& b, int steps, int& parity, double best, hipEvent_t e0, hipEvent_t e1) {
    enqueue_batch_chunk(b, 1, parity, false);
    parity ^= 1;
    auto timed = [&](int k) {
        FDLB_HIP(hipEventRecord(e0, b.stream));
        enqueue_batch_chunk(b, k, parity, false);
        if (k & 1) parity ^= 1;
        FDLB_HIP(hipEventRecord(e1, b.stream));
        FDLB_HIP(hipEventSynchronize(e1));
        float ms = 0;
        FDLB_HIP(hipEventElapsedTime(&ms, e0, e1));
        return (double)ms / k;
    };
    const double first = timed(1);
    if (first > 2.0 * best) return first;
    return timed(steps);
}

// Every member at rest (as fdlb_batch_init_equilibrium with no fields), one wait for all.
static void reseed_all(fdlb_batch& b) {
    for (auto& p : b.probs) init_rest_async(*p);
    FDLB_HIP(hipStreamSynchronize(b.stream));
}

// The shape a batch keeps, from the full-batch step times of the shapes timed: among those within
// 5 % of the fastest, the one that splits a tile's velocities over the most waves (then the
// faster).  A batch shrinks as its members converge, and the later, smaller launches pack short
// blocks better than long ones: on the 64-cavity sweep the four-way 64x8 tile, 3 % behind the
// two-way one on the full batch, solves the whole sweep 3-5 % sooner.
static int pick_batch_shape(int prec, const std::vector<std::pair<int, double>>& timed, double& ms_out) {
    double best = 1e300;
    for (const auto& tm : timed) best = std::min(best, tm.second);
    int pick = -1;
    double pick_ms = 0;
    for (const auto& tm : timed) {
        if (tm.second > 1.05 * best) continue;
        const int wa = tile_shapes(prec)[tm.first].wa;
        const int pwa = pick < 0 ? 0 : tile_shapes(prec)[pick].wa;
        if (pick < 0 || wa > pwa || (wa == pwa && tm.second < pick_ms)) {
            pick = tm.first;
            pick_ms = tm.second;
        }
    }
    ms_out = pick_ms;
    return pick;
}

// reseed: put the members back at rest at the end (the double group's pass, when it follows,
// re-seeds them itself).
double batch_autotune(fdlb_batch& b, int steps, bool reseed) {
    if (!b.bound) throw Error(FDLB_ESTATE, "batch is not bound to device memory");
    if (steps < 1) throw Error(FDLB_EINVAL, "steps must be >= 1");
    hipEvent_t e0, e1;
    FDLB_HIP(hipEventCreate(&e0));
    FDLB_HIP(hipEventCreate(&e1));
    const int g = primary_group(b);
    double best = 1e300;
    int best_tile = b.grp[g].tile;
    std::vector<std::pair<int, double>> timed;
    // Seeded once (every member in the primary group's precision): a step's cost does not depend
    // on the values it marches, so the shapes are timed one after another on the evolving state,
    // with the step parity carried over, and the members are re-seeded once at the end.
    reseed_all(b);
    int parity = 0;
    try {
        for (int t = 0; t < (int)tile_shapes(prec_of_group(g)).size(); ++t) {
            if (!tile_fits_all(b, g, t)) continue;
            group_set_tile(b, g, t);
            upload_args(b);
            b.active.clear();
            for (size_t i = 0; i < b.probs.size(); ++i) b.active.push_back((int)i);
            upload_map(b);
            const double ms = time_batch_shape(b, steps, parity, best, e0, e1);
            timed.emplace_back(t, ms);
            best = std::min(best, ms);
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!timed.empty()) best_tile = pick_batch_shape(prec_of_group(g), timed, best);
    group_set_tile(b, g, best_tile);
    if (reseed) reseed_all(b);
    return best;
}

// Tile of a mixed batch's double group: every member promoted (once), each fitting shape timed
// over `steps` steps of the whole batch on the evolving state (members re-seeded afterwards,
// back in float).
static void batch_autotune_promoted(fdlb_batch& b, int steps) {
    if (b.precision != FDLB_MIXED || !b.grp[1].used) return;
    hipEvent_t e0, e1;
    FDLB_HIP(hipEventCreate(&e0));
    FDLB_HIP(hipEventCreate(&e1));
    double best = 1e300;
    int best_tile = b.grp[1].tile;
    std::vector<std::pair<int, double>> timed;
    reseed_all(b);
    for (auto& p : b.probs) promote_async(*p);
    FDLB_HIP(hipStreamSynchronize(b.stream));
    int parity = 0;
    try {
        for (int t = 0; t < (int)tile_shapes(FDLB_FP64).size(); ++t) {
            if (!tile_fits_all(b, 1, t)) continue;
            group_set_tile(b, 1, t);
            upload_args(b);
            b.active.clear();
            for (size_t i = 0; i < b.probs.size(); ++i) b.active.push_back((int)i);
            upload_map(b);
            const double ms = time_batch_shape(b, steps, parity, best, e0, e1);
            timed.emplace_back(t, ms);
            best = std::min(best, ms);
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // (the double group holds only the members near convergence, a few at a time)
    if (!timed.empty()) best_tile = pick_batch_shape(FDLB_FP64, timed, best);
    group_set_tile(b, 1, best_tile);
    reseed_all(b);
}

}  // namespace fdlb

// ---- C ABI -------------------------------------------------------------------------------
namespace fdlb {
int guard_call(const std::function<int()>& f);
}

using namespace fdlb;

extern "C" {

int fdlb_batch_create(const fdlb_problem_desc* descs, int n, fdlb_batch** out) {
    return guard_call([&] {
        if (!out) throw Error(FDLB_EINVAL, "NULL output handle");
        *out = nullptr;
        auto b = std::make_unique<fdlb_batch>();
        batch_create(*b, descs, n);
        *out = b.release();
        return FDLB_OK;
    });
}

void fdlb_batch_destroy(fdlb_batch* b) { delete b; }

size_t fdlb_batch_state_bytes(const fdlb_batch* b) { return b ? b->state_bytes : 0; }
size_t fdlb_batch_workspace_bytes(const fdlb_batch* b) { return b ? b->work_bytes : 0; }

static fdlb_batch& bh(fdlb_batch* b) {
    if (!b) throw Error(FDLB_EINVAL, "NULL batch handle");
    return *b;
}

int fdlb_batch_bind(fdlb_batch* b, void* d_state, void* d_workspace, void* stream) {
    return guard_call([&] {
        batch_bind(bh(b), d_state, d_workspace, stream);
        return FDLB_OK;
    });
}

int fdlb_batch_init_equilibrium(fdlb_batch* b, int i, const double* rho, const double* ux, const double* uy,
                                int renormalize_mass) {
    return guard_call([&] {
        batch_init_equilibrium(bh(b), i, rho, ux, uy, renormalize_mass);
        return FDLB_OK;
    });
}

int fdlb_batch_init_equilibrium_dev(fdlb_batch* b, int i, const float* d_rho, const float* d_ux, const float* d_uy,
                                    int renormalize_mass) {
    return guard_call([&] {
        batch_init_equilibrium_dev(bh(b), i, d_rho, d_ux, d_uy, renormalize_mass);
        return FDLB_OK;
    });
}

int fdlb_batch_solve(fdlb_batch* b, double tol, int64_t max_steps, int32_t check_every, int32_t use_graph,
                     fdlb_report* reports) {
    return guard_call([&] { return batch_solve(bh(b), tol, max_steps, check_every, use_graph, reports); });
}

int fdlb_batch_moments(fdlb_batch* b, int i, double* rho, double* ux, double* uy, double* pxy) {
    return guard_call([&] {
        batch_moments(bh(b), i, rho, ux, uy, pxy);
        return FDLB_OK;
    });
}

int fdlb_batch_wall_profile(fdlb_batch* b, int i, int wall, double* rho, double* u_t, double* pxy) {
    return guard_call([&] {
        batch_wall_profile(bh(b), i, wall, rho, u_t, pxy);
        return FDLB_OK;
    });
}

int fdlb_batch_state_download(fdlb_batch* b, int i, double* f_host) {
    return guard_call([&] {
        batch_state_download(bh(b), i, f_host);
        return FDLB_OK;
    });
}

int fdlb_batch_state_upload(fdlb_batch* b, int i, const double* f_host) {
    return guard_call([&] {
        batch_state_upload(bh(b), i, f_host);
        return FDLB_OK;
    });
}

int fdlb_batch_field_samples(fdlb_batch* b, int i, float* d_in, float* d_target) {
    return guard_call([&] {
        field_samples(inst(bh(b), i), d_in, d_target);
        return FDLB_OK;
    });
}

int fdlb_batch_set_tile(fdlb_batch* b, int tile) {
    return guard_call([&] {
        batch_set_tile(bh(b), tile);
        return FDLB_OK;
    });
}

int fdlb_batch_set_retile(fdlb_batch* b, int max_members) {
    return guard_call([&] {
        if (max_members < 0) throw Error(FDLB_EINVAL, "max_members must be >= 0");
        bh(b).retile_members = max_members;
        return FDLB_OK;
    });
}

int fdlb_batch_set_pseudo_time(fdlb_batch* b, int on) {
    return guard_call([&] {
        fdlb_batch& B = bh(b);
        B.pseudo = on != 0;
        for (auto& p : B.probs) p->pseudo = on != 0;  // the next solve uploads the step arguments
        return FDLB_OK;
    });
}

int fdlb_batch_get_tile(const fdlb_batch* b) { return b ? b->grp[primary_group(*b)].tile : FDLB_EINVAL; }

int fdlb_batch_problem_q(const fdlb_batch* b, int i) {
    if (!b || i < 0 || i >= (int)b->probs.size()) return FDLB_EINVAL;
    return b->probs[i]->q;
}

int fdlb_batch_active_precision(const fdlb_batch* b, int i) {
    if (!b || i < 0 || i >= (int)b->probs.size()) return FDLB_EINVAL;
    return b->probs[i]->prec;
}

int fdlb_batch_autotune(fdlb_batch* b, int steps, double* best_ms_per_step) {
    return guard_call([&] {
        fdlb_batch& B = bh(b);
        std::string key;
        if (tune_cache_enabled()) {
            // the batch's whole make-up: every member's grid, velocity count and axes
            std::string members;
            for (auto& p : B.probs)
                members += std::to_string(p->d.nx) + "x" + std::to_string(p->d.ny) + "q" + std::to_string(p->q) +
                           (p->d.periodic_x ? "p" : "") + (p->d.periodic_y ? "P" : "") + ",";
            uint64_t h = 1469598103934665603ULL;
            for (char c : members) h = (h ^ (unsigned char)c) * 1099511628211ULL;
            char hx[32];
            std::snprintf(hx, sizeof(hx), "%016llx", (unsigned long long)h);
            key = tune_key_prefix() + "/batch/prec" + std::to_string(B.precision) + "/n" +
                  std::to_string(B.probs.size()) + "/" + hx;
            int t = -1, ta = -1;
            double ms = 0;
            if (B.bound && tune_cache_get(key, t, ta, ms)) {
                const int g = primary_group(B);
                const bool ok = t < (int)tile_shapes(prec_of_group(g)).size() && tile_fits_all(B, g, t) &&
                                (ta < 0 || !B.grp[1].used || g == 1 ||
                                 (ta < (int)tile_shapes(FDLB_FP64).size() && tile_fits_all(B, 1, ta)));
                if (ok) {
                    group_set_tile(B, g, t);
                    if (ta >= 0 && B.grp[1].used && g != 1) group_set_tile(B, 1, ta);
                    reseed_all(B);
                    if (best_ms_per_step) *best_ms_per_step = ms;
                    return FDLB_OK;
                }
            }
        }
        const bool promoted = B.precision == FDLB_MIXED && B.grp[1].used;
        const double ms = batch_autotune(B, steps, !promoted);
        batch_autotune_promoted(B, steps);
        if (!key.empty())
            tune_cache_put(key, B.grp[primary_group(B)].tile,
                           B.precision == FDLB_MIXED && B.grp[1].used ? B.grp[1].tile : -1, ms);
        if (best_ms_per_step) *best_ms_per_step = ms;
        return FDLB_OK;
    });
}

}  // extern "C"
