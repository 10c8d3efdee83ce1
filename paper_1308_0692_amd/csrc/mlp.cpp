// Host runtime of the warm-start network: layout of the parameter vector and the workspace,
// parameter initialisation, and the training / inference entry points of include/fdlb.h.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <memory>

#include "fdlb_internal.h"

struct fdlb_mlp {
    int hidden = 4;
    int P = 0;
    int64_t max_batch = 0;
    int64_t n_cap = 0;  // samples per layer of the bf16 transposes: max_batch rounded up to a slice
    int64_t nb_cap = 0; // training blocks of a full batch
    int32_t off_w[fdlb::MLP_MAX_HIDDEN + 1]{}, off_b[fdlb::MLP_MAX_HIDDEN + 1]{};
    size_t off_wbf = 0, off_wbfT = 0, off_hT = 0, off_dzT = 0, off_partw = 0, off_partt = 0, off_lossp = 0,
           off_loss = 0;
    size_t work_bytes = 0;
    float *params = nullptr, *grad = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    char* work = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    bool have_loss = false;
    double* pinned = nullptr;
    ~fdlb_mlp() {
        if (pinned) (void)hipHostFree(pinned);
    }
};

namespace fdlb {
int guard_call(const std::function<int()>& f);

namespace {
size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

fdlb_mlp& mh(fdlb_mlp* m) {
    if (!m) throw Error(FDLB_EINVAL, "NULL network handle");
    return *m;
}
void require_bound(const fdlb_mlp& m) {
    if (!m.bound) throw Error(FDLB_ESTATE, "network is not bound to device memory (call fdlb_mlp_bind)");
}

MlpArgs base_args(fdlb_mlp& m) {
    MlpArgs a;
    std::memset(&a, 0, sizeof(a));
    a.params = m.params;
    a.wbf = (const uint16_t*)(m.work + m.off_wbf);
    a.wbfT = (const uint16_t*)(m.work + m.off_wbfT);
    a.hidden = m.hidden;
    a.P = m.P;
    for (int l = 0; l <= m.hidden; ++l) {
        a.off_w[l] = m.off_w[l];
        a.off_b[l] = m.off_b[l];
    }
    return a;
}

// Refresh the bf16 copies of the hidden weights from the current parameters.
void refresh_bf16(fdlb_mlp& m, const MlpArgs& a) {
    launch_mlp_weights_bf16(a, (uint16_t*)(m.work + m.off_wbf), (uint16_t*)(m.work + m.off_wbfT), m.stream);
}

// splitmix64 (Steele, Lea & Flood 2014): a counter-based 64-bit generator.
uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}
}  // namespace

void mlp_create(fdlb_mlp& m, int hidden, int64_t max_batch) {
    if (hidden < 1 || hidden > MLP_MAX_HIDDEN) throw Error(FDLB_EINVAL, "hidden layers must be 1..8");
    if (max_batch < 1 || max_batch > ((int64_t)1 << 22)) throw Error(FDLB_EINVAL, "max_batch must be 1..2^22");
    m.hidden = hidden;
    m.max_batch = max_batch;
    int k = 0;
    for (int l = 0; l <= hidden; ++l) {
        const int out = l == hidden ? 3 : MLP_WIDTH;
        const int in = l == 0 ? 3 : MLP_WIDTH;
        m.off_w[l] = k;
        k += out * in;
        m.off_b[l] = k;
        k += out;
    }
    m.P = k;
    m.n_cap = (max_batch + MLP_SLICE - 1) / MLP_SLICE * MLP_SLICE;
    m.nb_cap = (max_batch + MLP_TRAIN_TILE - 1) / MLP_TRAIN_TILE;
    const size_t hw = (size_t)(hidden - 1) * MLP_WIDTH * MLP_WIDTH;
    const size_t tr = (size_t)(hidden - 1) * MLP_WIDTH * m.n_cap * sizeof(uint16_t);
    size_t off = 0;
    m.off_wbf = off;
    off += align256(hw * sizeof(uint16_t));
    m.off_wbfT = off;
    off += align256(hw * sizeof(uint16_t));
    m.off_hT = off;
    off += align256(tr);
    m.off_dzT = off;
    off += align256(tr);
    m.off_partw = off;
    off += align256((size_t)(m.n_cap / MLP_SLICE) * hw * sizeof(float));
    m.off_partt = off;
    off += align256((size_t)mlp_thin_count(hidden) * m.nb_cap * sizeof(float));
    m.off_lossp = off;
    off += align256((size_t)m.nb_cap * sizeof(double));
    m.off_loss = off;
    off += 256;
    m.work_bytes = off;
}

}  // namespace fdlb

using namespace fdlb;

// One training evaluation (forward, loss, gradient) of n samples; rows may be NULL.  The bf16
// weight copies are refreshed from the parameters unless the caller knows them current (the
// Adam update of the previous step of fdlb_mlp_train wrote them); with `adam`, the gradient
// reduction applies that Adam step too.
static void backward_of(fdlb_mlp& M, const float* d_in, const float* d_target, const int32_t* d_rows, int64_t n,
                        bool refresh = true, const AdamArgs* adam = nullptr) {
    require_bound(M);
    if (n < 1 || n > M.max_batch) throw Error(FDLB_EINVAL, "n must be 1..max_batch");
    if (!d_in || !d_target) throw Error(FDLB_EINVAL, "NULL input or target");
    MlpArgs a = base_args(M);
    a.in = d_in;
    a.target = d_target;
    a.rows = d_rows;
    a.n = n;
    a.n_cap = M.n_cap;
    a.nb_cap = M.nb_cap;
    a.hT = (uint16_t*)(M.work + M.off_hT);
    a.dzT = (uint16_t*)(M.work + M.off_dzT);
    a.part_w = (float*)(M.work + M.off_partw);
    a.part_thin = (float*)(M.work + M.off_partt);
    a.loss_part = (double*)(M.work + M.off_lossp);
    a.inv_3n = (float)(1.0 / (3.0 * (double)n));
    if (refresh) refresh_bf16(M, a);
    launch_mlp_train(a, M.stream);
    launch_mlp_wgrad(a, M.stream);
    launch_mlp_reduce(a, M.grad, 1.0 / (3.0 * (double)n), (double*)(M.work + M.off_loss), adam, M.stream);
    M.have_loss = true;
}

static void check_adam(double lr, double beta1, double beta2, double eps, int64_t step) {
    if (step < 1) throw Error(FDLB_EINVAL, "step counts from 1");
    if (!(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        throw Error(FDLB_EINVAL, "bad Adam hyper-parameters");
}

// Adam step `step` (from 1) of the bound parameters.
static AdamArgs adam_args(fdlb_mlp& M, double lr, double beta1, double beta2, double eps, int64_t step) {
    AdamArgs d;
    d.p = M.params;
    d.m = M.adam_m;
    d.v = M.adam_v;
    d.lr = (float)lr;
    d.b1 = (float)beta1;
    d.b2 = (float)beta2;
    d.eps = (float)eps;
    d.c1 = (float)(1.0 / (1.0 - std::pow(beta1, (double)step)));
    d.c2 = (float)(1.0 / (1.0 - std::pow(beta2, (double)step)));
    d.wbf = (uint16_t*)(M.work + M.off_wbf);
    d.wbfT = (uint16_t*)(M.work + M.off_wbfT);
    return d;
}

static void adam_of(fdlb_mlp& M, double lr, double beta1, double beta2, double eps, int64_t step) {
    launch_mlp_adam(base_args(M), M.grad, adam_args(M, lr, beta1, beta2, eps, step), M.stream);
}

extern "C" {

int fdlb_mlp_create(int hidden_layers, int64_t max_batch, fdlb_mlp** out) {
    return guard_call([&] {
        if (!out) throw Error(FDLB_EINVAL, "NULL output handle");
        *out = nullptr;
        auto m = std::make_unique<fdlb_mlp>();
        mlp_create(*m, hidden_layers, max_batch);
        *out = m.release();
        return FDLB_OK;
    });
}

void fdlb_mlp_destroy(fdlb_mlp* m) { delete m; }

int64_t fdlb_mlp_param_count(const fdlb_mlp* m) { return m ? m->P : FDLB_EINVAL; }
size_t fdlb_mlp_workspace_bytes(const fdlb_mlp* m) { return m ? m->work_bytes : 0; }

int fdlb_mlp_init_params(const fdlb_mlp* m, uint64_t seed, float* host_params) {
    return guard_call([&] {
        if (!m || !host_params) throw Error(FDLB_EINVAL, "NULL argument");
        uint64_t ctr = seed * 0x100000001b3ull;
        for (int l = 0; l <= m->hidden; ++l) {
            const int out = l == m->hidden ? 3 : MLP_WIDTH;
            const int in = l == 0 ? 3 : MLP_WIDTH;
            const double lim = std::sqrt(6.0 / (in + out));
            for (int e = 0; e < out * in; ++e) {
                const double u = (double)(splitmix64(ctr++) >> 11) * 0x1.0p-53;
                host_params[m->off_w[l] + e] = (float)(lim * (2.0 * u - 1.0));
            }
            for (int e = 0; e < out; ++e) host_params[m->off_b[l] + e] = 0.0f;
        }
        return FDLB_OK;
    });
}

int fdlb_mlp_bind(fdlb_mlp* m, float* d_params, float* d_grad, float* d_adam_m, float* d_adam_v, void* d_workspace,
                  void* stream) {
    return guard_call([&] {
        fdlb_mlp& M = mh(m);
        if (!d_params || !d_grad || !d_adam_m || !d_adam_v || !d_workspace)
            throw Error(FDLB_EINVAL, "device buffers must not be NULL");
        if ((uintptr_t)d_workspace & 255) throw Error(FDLB_EINVAL, "workspace must be 256-byte aligned");
        if (((uintptr_t)d_params | (uintptr_t)d_grad | (uintptr_t)d_adam_m | (uintptr_t)d_adam_v) & 3)
            throw Error(FDLB_EINVAL, "parameter buffers must be 4-byte aligned");
        M.params = d_params;
        M.grad = d_grad;
        M.adam_m = d_adam_m;
        M.adam_v = d_adam_v;
        M.work = (char*)d_workspace;
        M.stream = (hipStream_t)stream;
        if (!M.pinned) FDLB_HIP(hipHostMalloc((void**)&M.pinned, 8 * sizeof(double), hipHostMallocDefault));
        M.bound = true;
        M.have_loss = false;
        return FDLB_OK;
    });
}

int fdlb_mlp_forward(fdlb_mlp* m, const float* d_in, int64_t n, float* d_out) {
    return guard_call([&] {
        fdlb_mlp& M = mh(m);
        require_bound(M);
        if (n < 0) throw Error(FDLB_EINVAL, "n must be >= 0");
        if (n > 0 && (!d_in || !d_out)) throw Error(FDLB_EINVAL, "NULL input or output");
        MlpArgs a = base_args(M);
        a.in = d_in;
        a.out = d_out;
        a.n = n;
        refresh_bf16(M, a);
        launch_mlp_forward(a, M.stream);
        return FDLB_OK;
    });
}

int fdlb_mlp_backward(fdlb_mlp* m, const float* d_in, const float* d_target, const int32_t* d_rows, int64_t n) {
    return guard_call([&] {
        backward_of(mh(m), d_in, d_target, d_rows, n);
        return FDLB_OK;
    });
}

int fdlb_mlp_last_loss(fdlb_mlp* m, double* loss) {
    return guard_call([&] {
        fdlb_mlp& M = mh(m);
        require_bound(M);
        if (!loss) throw Error(FDLB_EINVAL, "NULL output");
        if (!M.have_loss) throw Error(FDLB_ESTATE, "no backward pass since binding");
        FDLB_HIP(hipMemcpyAsync(M.pinned, M.work + M.off_loss, sizeof(double), hipMemcpyDeviceToHost, M.stream));
        FDLB_HIP(hipStreamSynchronize(M.stream));
        *loss = M.pinned[0];
        return FDLB_OK;
    });
}

int fdlb_mlp_adam_step(fdlb_mlp* m, double lr, double beta1, double beta2, double eps, int64_t step) {
    return guard_call([&] {
        fdlb_mlp& M = mh(m);
        require_bound(M);
        check_adam(lr, beta1, beta2, eps, step);
        adam_of(M, lr, beta1, beta2, eps, step);
        return FDLB_OK;
    });
}

int fdlb_mlp_train(fdlb_mlp* m, const float* d_in, const float* d_target, const int32_t* d_rows, int64_t n_rows,
                   int64_t batch, int64_t steps, const double* lr, double beta1, double beta2, double eps,
                   int64_t first_step) {
    return guard_call([&] {
        fdlb_mlp& M = mh(m);
        require_bound(M);
        if (!d_in || !d_target || !d_rows || (steps > 0 && !lr)) throw Error(FDLB_EINVAL, "NULL array");
        if (batch < 1 || batch > M.max_batch) throw Error(FDLB_EINVAL, "batch must be 1..max_batch");
        // step s starts at row s * batch: the last one must start before n_rows (no overflow)
        if (steps < 0 || n_rows < 0 || (steps > 0 && (n_rows < 1 || steps - 1 > (n_rows - 1) / batch)))
            throw Error(FDLB_EINVAL, "every step needs at least one row");
        for (int64_t s = 0; s < steps; ++s) check_adam(lr[s], beta1, beta2, eps, first_step + s);
        for (int64_t s = 0; s < steps; ++s) {
            const int64_t r0 = s * batch, n = std::min(batch, n_rows - r0);
            // the reduction of the gradient applies the update as it goes (the same arithmetic
            // as fdlb_mlp_adam_step)
            const AdamArgs d = adam_args(M, lr[s], beta1, beta2, eps, first_step + s);
            backward_of(M, d_in, d_target, d_rows + r0, n, s == 0, &d);
        }
        return FDLB_OK;
    });
}

int fdlb_mlp_predict_fields(fdlb_mlp* m, double kn, int nx, int ny, double u_w, float* d_rho, float* d_ux,
                            float* d_uy) {
    return guard_call([&] {
        fdlb_mlp& M = mh(m);
        require_bound(M);
        if (!(kn > 0) || !std::isfinite(kn)) throw Error(FDLB_EINVAL, "kn must be positive and finite");
        if (!std::isfinite(u_w)) throw Error(FDLB_EINVAL, "u_w must be finite");
        if (nx < 1 || ny < 1) throw Error(FDLB_EINVAL, "nx and ny must be >= 1");
        if (!d_rho || !d_ux || !d_uy) throw Error(FDLB_EINVAL, "NULL output field");
        MlpArgs a = base_args(M);
        a.n = (int64_t)nx * ny;
        a.cells_nx = nx;
        a.cells_ny = ny;
        a.kn_feat = mlp_kn_feature(kn);
        a.u_w = (float)u_w;
        a.f_rho = d_rho;
        a.f_ux = d_ux;
        a.f_uy = d_uy;
        refresh_bf16(M, a);
        launch_mlp_forward(a, M.stream);
        return FDLB_OK;
    });
}

}  // extern "C"
