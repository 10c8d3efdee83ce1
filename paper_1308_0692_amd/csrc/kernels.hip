// Device kernels of libfdlb for gfx950 (CDNA4, wave64).
//
// State: populations in structure-of-arrays planes h[alpha][y][x].  The FP64
// path stores h = f_alpha - w_alpha in double, the FP32 path in float; the
// change of variable is exact because the scheme is linear and the rest
// state f_alpha = w_alpha is a fixed point of it (Eqs. 1, 5, 8-9).
//
// One time step (the fully discrete scheme: explicit-Euler relaxation, then
// first-order upwind transport) is ONE pass of step_kernel over the state:
// every population is read once and written once.  The relaxation needs the
// density and momentum of each cell over all velocities (Eqs. 6-7), and the
// wall emission needs the impermeability sum of Eq. (9) over the arriving
// half of the wall cell's relaxed populations; both are accumulated while
// the previous step writes its output and read back at the start of the
// next, so no second pass over the state is needed:
//   sum over arriving xi of |xi_n| g = (1-omega) Phi + omega (rho_h A + j_n Bn + j_t Bt)
// with Phi the same sum over h (kept in double) and A, Bn, Bt constants of
// the velocity set.
//
// Work decomposition: a wave owns a tile of (LX*VX) x (LY*K) cells (LX lanes
// along x, LY = 64/LX along y, each lane VX consecutive cells of K rows) and
// loops over the velocities quadrant by quadrant (signs of xi_x, xi_y are
// then compile-time constants); small grids split the velocities of a tile
// over 2, 4 or 8 waves whose partial moments meet in LDS.  The upwind
// neighbour of a cell is in the same lane's registers, in a neighbouring lane
// (cross-lane shuffle of the relaxed value), in a halo cell outside the wave
// (loaded and relaxed by the edge lane), or the wall emission of Eq. (8).
// Blocks are mapped to tiles so that each of the 8 XCDs owns a contiguous band
// of tile rows, keeping vertically adjacent tiles, which read each other's edge
// rows as halos, on one XCD and its L2.
//
// Residual: every block writes three partial sums; they are reduced by a
// one-block kernel after the step (large grids) or by one extra block of the
// next step's launch (grids of at most INLINE_REDUCE_MAX_BLOCKS tiles), in a
// fixed order either way, so runs are bit-reproducible.
#include <algorithm>
#include <type_traits>

#include "fdlb_internal.h"

namespace fdlb {

namespace {

constexpr int NUM_XCD = 8;

#ifdef FDLB_MIN_WAVES  // ask the register allocator for this many waves per SIMD
#define FDLB_WAVES_ATTR __attribute__((amdgpu_waves_per_eu(FDLB_MIN_WAVES)))
#else
#define FDLB_WAVES_ATTR
#endif

enum : int { MODE_SHUF = 0, MODE_LOAD = 1, MODE_WALL = 2 };

// Tile index of a block so that XCD k (blocks b with b % 8 == k) owns tiles
// [start_k, start_k + count_k): hardware dispatches blocks round-robin over XCDs.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int k = b % NUM_XCD, i = b / NUM_XCD;
    const int q = nb / NUM_XCD, r = nb % NUM_XCD;
    return k * q + (k < r ? k : r) + i;
}

template <int N, class T>
__device__ __forceinline__ void vload(T (&dst)[N], const T* p) {
    if constexpr (N == 1) {
        dst[0] = p[0];
    } else {
        typedef T V __attribute__((ext_vector_type(N)));
        const V v = *reinterpret_cast<const V*>(p);
#pragma unroll
        for (int i = 0; i < N; ++i) dst[i] = v[i];
    }
}

// Population stores, non-temporal for tiles that stream large grids (NT): the next read of a
// plane comes after the whole grid has been swept, so keeping it in L2 gains nothing there.
template <int N, bool NT, class T>
__device__ __forceinline__ void vstore_pop(T* p, const T (&src)[N]) {
    typedef T V __attribute__((ext_vector_type(N)));
    if constexpr (N == 1) {
        if constexpr (NT) __builtin_nontemporal_store(src[0], p);
        else p[0] = src[0];
    } else {
        V v;
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = src[i];
        if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<V*>(p));
        else *reinterpret_cast<V*>(p) = v;
    }
}

template <int N, class T>
__device__ __forceinline__ void vstore(T* p, const T (&src)[N]) {
    if constexpr (N == 1) {
        p[0] = src[0];
    } else {
        typedef T V __attribute__((ext_vector_type(N)));
        V v;
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = src[i];
        *reinterpret_cast<V*>(p) = v;
    }
}

// Velocity-table entries are read-only for the whole launch: reading them through the
// constant address space lets uniform indices use scalar loads.
template <class T>
__device__ __forceinline__ VelEntry<T> load_vel(const VelEntry<T>* p, const int e) {
    typedef const __attribute__((address_space(4))) VelEntry<T>* cptr;
    const cptr q = ((cptr)p) + e;
    VelEntry<T> v;
    v.ow = q->ow;
    v.owx = q->owx;
    v.owy = q->owy;
    v.w = q->w;
    v.wx = q->wx;
    v.wy = q->wy;
    v.xx = q->xx;
    v.xy = q->xy;
    v.nux = q->nux;
    v.nuy = q->nuy;
    v.alpha = q->alpha;
    v.pt = q->pt;
    return v;
}
template <class T>
__device__ __forceinline__ int load_alpha(const VelEntry<T>* p, const int e) {
    typedef const __attribute__((address_space(4))) VelEntry<T>* cptr;
    return ((cptr)p)[e].alpha;
}
template <class T>
__device__ __forceinline__ int64_t load_off(const VelEntry<T>* p, const int e) {
    typedef const __attribute__((address_space(4))) VelEntry<T>* cptr;
    return ((cptr)p)[e].off;
}

// The value v holds in lane (lane - D); lanes whose source lies outside the wave get a value
// that callers never use.  A shift by one lane is a DPP wave shift (a register move: no LDS
// round trip, no wait on the counter that LDS shares with scalar loads); other distances go
// through ds_bpermute.
template <int D, class T>
__device__ __forceinline__ T lane_from(const T v, const int lane) {
    if constexpr (D == 1 || D == -1) {
        constexpr int CTRL = D == 1 ? 0x138 : 0x130;  // wave_shr:1 (from lane - 1), wave_shl:1 (lane + 1)
        if constexpr (sizeof(T) == 4) {
            return __builtin_bit_cast(
                T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
        } else {
            const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
            const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
            const unsigned hi =
                (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
            return __builtin_bit_cast(T, ((unsigned long long)hi << 32) | lo);
        }
    } else {
        return __shfl(v, lane - D, 64);
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// The three residual sums of a step from its block partials, in one fixed order (lane l adds
// blocks l, l + 64, ...; then an xor butterfly, whose pairwise sums are the same on both lanes
// of a pair), so that every wave that calls it gets bit-identical totals.
__device__ __forceinline__ void wave_partials(const double* __restrict__ pp, int nb, double& num, double& den,
                                              double& umax2) {
    const int lane = threadIdx.x & 63;
    double a = 0.0, b = 0.0, m = 0.0;
    for (int i = lane; i < nb; i += 64) {
        a += pp[3 * i];
        b += pp[3 * i + 1];
        m = fmax(m, pp[3 * i + 2]);
    }
    num = wave_sum(a);
    den = wave_sum(b);
    umax2 = wave_max(m);
}

}  // namespace

// ---------------------------------------------------------------------------
// The fused time step.
// ---------------------------------------------------------------------------
// A problem whose solve has converged or diverged stops being updated (its state stays at
// the step that met the criterion), when the control block asks for it.
__device__ __forceinline__ bool frozen(const double* __restrict__ ctrl) {
    // (bitwise, not short-circuit: the three loads are issued together, one round trip)
    const double f = ctrl[CTRL_FREEZE], a = ctrl[CTRL_FIRST_BELOW], d = ctrl[CTRL_DIVERGED];
    return (f != 0.0) & ((a >= 0.0) | (d >= 0.0));
}

// Residual of a step from its sums: R = sqrt(sum |du|^2 / sum |u|^2).  A state at rest that
// stays at rest has R = 0, one that leaves rest R = inf; a non-finite state makes the sums NaN
// and so R, which counts as a runaway (never as convergence).
__device__ __forceinline__ double residual_of(double num, double den) {
    if (den > 0.0) return sqrt(num / den);
    if (den == 0.0 && num == 0.0) return 0.0;
    if (den == 0.0 && num > 0.0) return __builtin_huge_val();
    return __builtin_nan("");
}
__device__ __forceinline__ bool runaway(double R, double umax2) { return !(R <= 1e300) || !(umax2 <= 0.25); }

// Step bookkeeping in the control block (one thread): counter, residual, ring, first step
// below the tolerance, first runaway step.
__device__ __forceinline__ void record_step(double* __restrict__ ctrl, double num, double den, double umax2,
                                            int64_t inc) {
    const double R = residual_of(num, den);
    const double step = ctrl[CTRL_STEP] + (double)inc;
    ctrl[CTRL_STEP] = step;
    ctrl[CTRL_LAST_R] = R;
    ctrl[CTRL_MAXU] = sqrt(umax2);
    ctrl[CTRL_RING + ((int64_t)step - 1) % CTRL_RING_LEN] = R;
    if (R < ctrl[CTRL_TOL] && ctrl[CTRL_FIRST_BELOW] < 0.0) ctrl[CTRL_FIRST_BELOW] = step;
    if (runaway(R, umax2) && ctrl[CTRL_DIVERGED] < 0.0) ctrl[CTRL_DIVERGED] = step;
}


// A block is WX x WPB x WA waves: WX waves side by side along x, WPB stacked along y, each
// replicated WA times along the velocity index (the partial moments of the WA waves are summed
// through LDS in a fixed order).  With WA a multiple of 4, wave wa takes the velocities of
// quadrant wa mod 4 only, every (WA/4)-th one, so that a wave meets one quadrant's first-load
// latency instead of four; otherwise it takes every WA-th velocity of each quadrant.
// bid/nb: this block's index among the blocks of its problem; part: where its residual
// partials go.
template <class T, int VX, int K, int LX, int WPB, int WA, int WX, bool NT, int PD, bool PS>
__device__ __forceinline__ void step_body(const StepArgs<T>& A, const int bid, const int nb,
                                          double* __restrict__ part) {
    constexpr int LY = 64 / LX;
    constexpr int WPT = WX * WPB;  // waves per tile
    const int lane = threadIdx.x & 63;
    // The wave index is uniform; saying so keeps everything derived from it (velocity-table
    // indices in particular) in scalar registers and scalar loads.
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wxi = wave % WX, wy = (wave / WX) % WPB, wa = wave / WPT;
    const int wt = wave % WPT;     // wave index within the tile
    const int lx = lane % LX, ly = lane / LX;
    const int tile = xcd_tile(bid, nb);
    const int tx = tile % A.tiles_x, ty = tile / A.tiles_x;
    const int nx = A.nx, ny = A.ny, L = A.L;
    const int64_t plane = A.plane;
    const int x0 = (tx * WX + wxi) * (LX * VX) + lx * VX;
    const int y0 = ((ty * WPB + wy) * LY + ly) * K;
    const bool xv = x0 < nx;
    const T om = A.omega;

    bool rv[K];  // row r of this lane is a cell of the grid
#pragma unroll
    for (int r = 0; r < K; ++r) rv[r] = xv && (y0 + r < ny);

    // Density and momentum (deviation form) of this lane's cells, from the previous step.
    // They are carried in double; the relaxation uses them rounded to the storage type.
    T mr[K][VX], mx[K][VX], my[K][VX];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        if (rv[r]) {
            const int64_t o = (int64_t)(y0 + r) * nx + x0;
            double t0[VX], t1[VX], t2[VX];
            vload<VX>(t0, A.mom_in + o);
            vload<VX>(t1, A.mom_in + plane + o);
            vload<VX>(t2, A.mom_in + 2 * plane + o);
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                mr[r][v] = (T)t0[v];
                mx[r][v] = (T)t1[v];
                my[r][v] = (T)t2[v];
            }
        } else {
#pragma unroll
            for (int v = 0; v < VX; ++v) mr[r][v] = mx[r][v] = my[r][v] = T(0);
        }
    }
    // Checked after the moment loads are issued, so that the control-block read overlaps them
    // (the whole block takes the same branch: the control block is uniform).
    if (frozen(A.ctrl)) return;

    // Wall emission parameters of this step (Eqs. 8-9): rho_w - 1 and u_w rho_w per wall face.
    const double omega = A.omega_d;
    // (bitwise, not short-circuit: no branch, and no round trip, per wall flag)
    const bool on_left = xv & (x0 == 0) & (A.wall[LEFT].active != 0);
    const bool on_right = xv & (x0 + VX == nx) & (A.wall[RIGHT].active != 0);
    const bool on_bot = xv & (y0 == 0) & (A.wall[BOTTOM].active != 0);
    const int r_top = ny - 1 - y0;
    const bool on_top = xv & (r_top >= 0) & (r_top < K) & (A.wall[TOP].active != 0);
    const int xw = on_left ? LEFT : RIGHT;
    const int yw = on_bot ? BOTTOM : TOP;

    T Px[K], Qx[K];
    double phx[K];
#pragma unroll
    for (int r = 0; r < K; ++r) {
        Px[r] = Qx[r] = T(0);
        phx[r] = 0.0;
    }
    if (on_left || on_right) {
        const WallConst W = A.wall[xw];
        const int vi = on_left ? 0 : VX - 1;
        const double sn = on_left ? 1.0 : -1.0;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            if (rv[r]) {
                const double phi = A.phi_in[xw * L + y0 + r];
                const int64_t o = (int64_t)(y0 + r) * nx + x0 + vi;
                const double s = (1.0 - omega) * phi +
                                 omega * (A.mom_in[o] * W.A + sn * A.mom_in[plane + o] * W.Bn +
                                          A.mom_in[2 * plane + o] * W.Bt);
                const double P = W.c0 + W.k * s;
                Px[r] = (T)P;
                Qx[r] = (T)(W.u * (1.0 + P));
            }
        }
    }
    T Py[VX], Qy[VX];
    double phy[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        Py[v] = Qy[v] = T(0);
        phy[v] = 0.0;
    }
    if (on_bot || on_top) {
        const WallConst W = A.wall[yw];
        const double sn = on_bot ? 1.0 : -1.0;
        const int rw = on_bot ? 0 : r_top;
#pragma unroll
        for (int v = 0; v < VX; ++v) {
            const int64_t o = (int64_t)(y0 + rw) * nx + x0 + v;
            const double wr = A.mom_in[o], wx = A.mom_in[plane + o], wy = A.mom_in[2 * plane + o];
            const double phi = A.phi_in[yw * L + x0 + v];
            const double s = (1.0 - omega) * phi + omega * (wr * W.A + sn * wy * W.Bn + wx * W.Bt);
            const double P = W.c0 + W.k * s;
            Py[v] = (T)P;
            Qy[v] = (T)(W.u * (1.0 + P));
        }
    }
    const int r_top_in = (r_top >= 0 && r_top < K - 1) ? r_top : -1;

    // Moments of the new state, accumulated over all velocities in double (a float sum of
    // terms dominated by the even part w rho_h would carry ~1e-7 relative noise into the
    // momentum and hence into the residual).
    double ar[K][VX], ax[K][VX], ay[K][VX];
#pragma unroll
    for (int r = 0; r < K; ++r)
#pragma unroll
        for (int v = 0; v < VX; ++v) ar[r][v] = ax[r][v] = ay[r][v] = 0.0;

    auto quadrant = [&](auto sxc, auto syc, const int qb, const int qe) {
        constexpr int SX = decltype(sxc)::value;
        constexpr int SY = decltype(syc)::value;
        constexpr int QI = (SX < 0 ? 1 : 0) + (SY < 0 ? 2 : 0);  // quadrant order of the table
        constexpr bool QSPLIT = WA % 4 == 0;
        constexpr int SW = QSPLIT ? WA / 4 : WA;  // stride between this wave's planes
        if (QSPLIT && (wa & 3) != QI) return;
        // Where the lane-boundary cell's upwind neighbour comes from.
        int xmode, xh;
        if constexpr (SX > 0) {
            xh = x0 - 1;
            xmode = (x0 == 0) ? MODE_WALL : (lx > 0 ? MODE_SHUF : MODE_LOAD);
        } else {
            xh = x0 + VX;
            xmode = (x0 + VX >= nx) ? MODE_WALL : (lx < LX - 1 ? MODE_SHUF : MODE_LOAD);
        }
        int ymode, yh;
        if constexpr (SY > 0) {
            yh = y0 - 1;
            ymode = (y0 == 0) ? MODE_WALL : (ly > 0 ? MODE_SHUF : MODE_LOAD);
        } else {
            yh = y0 + K;
            ymode = (y0 + K >= ny) ? MODE_WALL : (ly < LY - 1 ? MODE_SHUF : MODE_LOAD);
        }
        // A lane with no cell of the grid loads nothing (its halo may lie outside the grid).
        if (!xv || y0 >= ny) xmode = ymode = MODE_WALL;
        // Moments of the halo cells this lane relaxes itself.
        T hxr[K], hxx[K], hxy[K];
#pragma unroll
        for (int r = 0; r < K; ++r) {
            hxr[r] = hxx[r] = hxy[r] = T(0);
            if (xmode == MODE_LOAD && rv[r]) {
                const int64_t o = (int64_t)(y0 + r) * nx + xh;
                hxr[r] = (T)A.mom_in[o];
                hxx[r] = (T)A.mom_in[plane + o];
                hxy[r] = (T)A.mom_in[2 * plane + o];
            }
        }
        T hyr[VX], hyx[VX], hyy[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) hyr[v] = hyx[v] = hyy[v] = T(0);
        if (ymode == MODE_LOAD) {
            const int64_t o = (int64_t)yh * nx + x0;
            double t0[VX], t1[VX], t2[VX];
            vload<VX>(t0, A.mom_in + o);
            vload<VX>(t1, A.mom_in + plane + o);
            vload<VX>(t2, A.mom_in + 2 * plane + o);
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                hyr[v] = (T)t0[v];
                hyx[v] = (T)t1[v];
                hyy[v] = (T)t2[v];
            }
        }

        // Plane e of the source.  Tiles with one or two cells per lane take the plane's byte offset
        // precomputed in the table: one 64-bit add instead of a 64-bit multiply on the scalar
        // unit, which the many small waves of such tiles keep busy (measured: 5-9 % per step on
        // 64^2-192^2 grids); wider tiles are bound by HBM and keep the multiply, with which
        // their loads issue best.
        constexpr bool OFF = K * VX <= 2;
        auto plane_of = [&](const T* base, const int e) -> const T* {
            if constexpr (OFF) return (const T*)((const char*)base + load_off(A.vel, e));
            else return base + (int64_t)load_alpha(A.vel, e) * plane;
        };
        // Loads of one velocity plane: this lane's cells and the halo cells it relaxes itself.
        // Every load is unconditional, from an address that is always inside the plane (rows
        // past the grid read its last row, a halo that is not needed reads the lane's own cell;
        // such values are never used): loads under divergent branches would force the
        // compiler to drain all outstanding loads, including the prefetched planes.
        int64_t orow[K], ohx[K];
        const int xc = xv ? x0 : 0;
        const int xhc = (xmode == MODE_LOAD) ? xh : xc;
#pragma unroll
        for (int r = 0; r < K; ++r) {
            const int yc = (y0 + r < ny) ? y0 + r : ny - 1;
            orow[r] = (int64_t)yc * nx + xc;
            ohx[r] = (int64_t)yc * nx + xhc;
        }
        const int64_t ohy = (int64_t)((ymode == MODE_LOAD) ? yh : (y0 < ny ? y0 : ny - 1)) * nx + xc;
        auto load_plane = [&](const int e, T (&hv)[K][VX], T (&hx)[K], T (&hy)[VX]) {
            const T* __restrict__ s = plane_of(A.src, e);
#pragma unroll
            for (int r = 0; r < K; ++r) vload<VX>(hv[r], s + orow[r]);
#pragma unroll
            for (int r = 0; r < K; ++r) hx[r] = s[ohx[r]];
            vload<VX>(hy, s + ohy);
        };

        // Software pipeline over velocities: the loads of the next PD planes of this wave are in
        // flight while the current one is relaxed, transported and stored (under load, one
        // plane's round trip to HBM lasts longer than the compute on it).  The loop is unrolled
        // PD + 1 times so that the plane buffers change roles without register copies (a copy
        // out of a buffer whose load is in flight would have to wait for it).
        static_assert(PD >= 1 && PD <= 8, "prefetch distance must be 1..8");
        const int e0 = qb + (QSPLIT ? (wa >> 2) : wa);
        const int elast = qe - 1 - ((qe - 1 - e0) % SW);  // last plane of this wave (if e0 < qe)
        auto clampe = [&](const int en) { return en <= elast ? en : elast; };

        auto step_one = [&](const int e, const T (&g)[K][VX], const T (&gxh_in)[K], const T (&gyh_in)[VX]) {
            const VelEntry<T> c = load_vel(A.vel, e);
            T* __restrict__ d = OFF ? (T*)((char*)A.dst + load_off(A.vel, e)) : A.dst + (int64_t)c.alpha * plane;
            T gxh[K], gyh[VX];
#pragma unroll
            for (int r = 0; r < K; ++r) gxh[r] = gxh_in[r];
#pragma unroll
            for (int v = 0; v < VX; ++v) gyh[v] = gyh_in[v];
            T gr[K][VX];

            // Relaxation (explicit Euler of Eq. 1 towards Eq. 5, deviation form).
            // g = h + (omega h_eq - omega h): the increment is formed before it is added, so the
            // relaxation rate is omega itself (a rounded 1 - omega would bias a small omega).
#pragma unroll
            for (int r = 0; r < K; ++r)
#pragma unroll
                for (int v = 0; v < VX; ++v)
                    gr[r][v] = g[r][v] + ((c.ow * mr[r][v] + c.owx * mx[r][v] + c.owy * my[r][v]) - om * g[r][v]);
#pragma unroll
            for (int r = 0; r < K; ++r)
                gxh[r] = gxh[r] + ((c.ow * hxr[r] + c.owx * hxx[r] + c.owy * hxy[r]) - om * gxh[r]);
#pragma unroll
            for (int v = 0; v < VX; ++v)
                gyh[v] = gyh[v] + ((c.ow * hyr[v] + c.owx * hyx[v] + c.owy * hyy[v]) - om * gyh[v]);

            // Upwind values across the lane boundary: neighbour lane, halo, or wall emission.
            T xb[K];
#pragma unroll
            for (int r = 0; r < K; ++r) {
                const T sh = lane_from<SX>(gr[r][SX > 0 ? VX - 1 : 0], lane);
                const T em = c.w * Px[r] + c.wy * Qx[r];
                xb[r] = xmode == MODE_SHUF ? sh : (xmode == MODE_LOAD ? gxh[r] : em);
            }
            T yb[VX];
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const T sh = lane_from<SY * LX>(gr[SY > 0 ? K - 1 : 0][v], lane);
                const T em = c.w * Py[v] + c.wx * Qy[v];
                yb[v] = ymode == MODE_SHUF ? sh : (ymode == MODE_LOAD ? gyh[v] : em);
            }

            // First-order upwind transport.
            T fn[K][VX];
#pragma unroll
            for (int r = 0; r < K; ++r) {
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const T gc = gr[r][v];
                    T gx, gy;
                    if constexpr (SX > 0) gx = (v > 0) ? gr[r][v - 1] : xb[r];
                    else gx = (v < VX - 1) ? gr[r][v + 1] : xb[r];
                    if constexpr (SY > 0) {
                        gy = (r > 0) ? gr[r - 1][v] : yb[v];
                    } else {
                        gy = (r < K - 1) ? gr[r + 1][v] : yb[v];
                        if (r == r_top_in) gy = c.w * Py[v] + c.wx * Qy[v];
                    }
                    fn[r][v] = gc - c.nux * (gc - gx) - c.nuy * (gc - gy);
                }
            }
            if constexpr (PS) {
                // Velocity-local pseudo-time steps (steady iterations only): the state moves by
                // pt times the step's change, h + pt (S h - h), which keeps the fixed point of S.
                // The change (relaxation increment minus the transport differences) is formed
                // again from its parts, not as S h - h, so that pt does not magnify the rounding
                // of S h.
                const T pt = (T)c.pt;
#pragma unroll
                for (int r = 0; r < K; ++r) {
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        const T gc = gr[r][v];
                        T gx, gy;
                        if constexpr (SX > 0) gx = (v > 0) ? gr[r][v - 1] : xb[r];
                        else gx = (v < VX - 1) ? gr[r][v + 1] : xb[r];
                        if constexpr (SY > 0) {
                            gy = (r > 0) ? gr[r - 1][v] : yb[v];
                        } else {
                            gy = (r < K - 1) ? gr[r + 1][v] : yb[v];
                            if (r == r_top_in) gy = c.w * Py[v] + c.wx * Qy[v];
                        }
                        const T inc = (c.ow * mr[r][v] + c.owx * mx[r][v] + c.owy * my[r][v]) - om * g[r][v];
                        fn[r][v] = g[r][v] + pt * ((inc - c.nux * (gc - gx)) - c.nuy * (gc - gy));
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < K; ++r)
                if (rv[r]) vstore_pop<VX, NT>(d + (int64_t)(y0 + r) * nx + x0, fn[r]);

            // Moments (Eqs. 6-7) and wall fluxes of the new state.
#pragma unroll
            for (int r = 0; r < K; ++r)
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const double fd = (double)fn[r][v];
                    ar[r][v] += fd;
                    ax[r][v] += (double)c.xx * fd;
                    ay[r][v] += (double)c.xy * fd;
                }
            if constexpr (SX < 0) {
                if (on_left) {
#pragma unroll
                    for (int r = 0; r < K; ++r) phx[r] += -(double)c.xx * (double)fn[r][0];
                }
            } else {
                if (on_right) {
#pragma unroll
                    for (int r = 0; r < K; ++r) phx[r] += (double)c.xx * (double)fn[r][VX - 1];
                }
            }
            if constexpr (SY < 0) {
                if (on_bot) {
#pragma unroll
                    for (int v = 0; v < VX; ++v) phy[v] += -(double)c.xy * (double)fn[0][v];
                }
            } else {
                if (on_top) {
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        T t = T(0);
#pragma unroll
                        for (int r = 0; r < K; ++r)
                            if (r == r_top) t = fn[r][v];
                        phy[v] += (double)c.xy * (double)t;
                    }
                }
            }
        };

        // Planes past this wave's last one are clamped to it: loaded again, never used.
        T bv[PD + 1][K][VX], bx[PD + 1][K], by[PD + 1][VX];
        if (e0 < qe) {
#pragma unroll
            for (int j = 0; j < PD; ++j) load_plane(clampe(e0 + j * SW), bv[j], bx[j], by[j]);
            for (int e = e0;;) {
#pragma unroll
                for (int j = 0; j <= PD; ++j) {
                    const int jl = (j + PD) % (PD + 1);  // the buffer that plane e + PD*SW goes to
                    load_plane(clampe(e + PD * SW), bv[jl], bx[jl], by[jl]);
                    step_one(e, bv[j], bx[j], by[j]);
                    if ((e += SW) >= qe) goto planes_done;
                }
            }
        planes_done:;
        }
    };

    quadrant(std::integral_constant<int, 1>{}, std::integral_constant<int, 1>{}, A.quad_begin[0],
             A.quad_begin[1]);
    quadrant(std::integral_constant<int, -1>{}, std::integral_constant<int, 1>{}, A.quad_begin[1],
             A.quad_begin[2]);
    quadrant(std::integral_constant<int, 1>{}, std::integral_constant<int, -1>{}, A.quad_begin[2],
             A.quad_begin[3]);
    quadrant(std::integral_constant<int, -1>{}, std::integral_constant<int, -1>{}, A.quad_begin[3],
             A.quad_begin[4]);

    double num = 0.0, den = 0.0, umax = 0.0;
    if constexpr (WA > 1) {
        // The WA waves that share this tile meet in LDS: every wave leaves its partial sums there,
        // and cell c = r VX + v of each lane is then summed (wave 0's partial first, then in
        // increasing wave order), written and checked by wave c % WA, the wall sums by wave 0.
        // The epilogue is spread over the tile's waves instead of running on one while the others
        // wait; the sums are the same whichever wave forms them.
        constexpr int NM = 3 * K * VX + K + VX;  // doubles per lane
        __shared__ double xred[WA][WPT][NM][64];
        {
            double* o = &xred[wa][wt][0][lane];
            int i = 0;
#pragma unroll
            for (int r = 0; r < K; ++r)
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    o[64 * i++] = ar[r][v];
                    o[64 * i++] = ax[r][v];
                    o[64 * i++] = ay[r][v];
                }
#pragma unroll
            for (int r = 0; r < K; ++r) o[64 * i++] = phx[r];
#pragma unroll
            for (int v = 0; v < VX; ++v) o[64 * i++] = phy[v];
        }
        __syncthreads();
        auto total = [&](const int i) {
            double t = xred[0][wt][i][lane];
#pragma unroll
            for (int w = 1; w < WA; ++w) t += xred[w][wt][i][lane];
            return t;
        };
#pragma unroll
        for (int r = 0; r < K; ++r)
#pragma unroll
            for (int v = 0; v < VX; ++v) {
                const int c = r * VX + v;
                if (c % WA != wa || !rv[r]) continue;
                const double sr = total(3 * c), sx = total(3 * c + 1), sy = total(3 * c + 2);
                const int64_t o = (int64_t)(y0 + r) * nx + x0 + v;
                A.mom_out[o] = sr;
                A.mom_out[plane + o] = sx;
                A.mom_out[2 * plane + o] = sy;
                // residual terms against the old moments, re-read; one double division per
                // cell: 1 / r0 = r1 / (r0 r1), 1 / r1 = r0 / (r0 r1)
                const double r0 = 1.0 + A.mom_in[o], r1 = 1.0 + sr;
                const double inv = 1.0 / (r0 * r1);
                const double i0 = r1 * inv, i1 = r0 * inv;
                const double ux0 = A.mom_in[plane + o] * i0, uy0 = A.mom_in[2 * plane + o] * i0;
                const double ux1 = sx * i1, uy1 = sy * i1;
                const double dx = ux1 - ux0, dy = uy1 - uy0;
                const double u2 = ux1 * ux1 + uy1 * uy1;
                num += dx * dx + dy * dy;
                den += u2;
                umax = fmax(umax, u2);
            }
        if (wa == 0) {
            if (on_left || on_right) {
#pragma unroll
                for (int r = 0; r < K; ++r)
                    if (rv[r]) A.phi_out[xw * L + y0 + r] = total(3 * K * VX + r);
            }
            if (on_bot || on_top) {
#pragma unroll
                for (int v = 0; v < VX; ++v) A.phi_out[yw * L + x0 + v] = total(3 * K * VX + K + v);
            }
        }
    } else {
        // Outputs for the next step.
#pragma unroll
        for (int r = 0; r < K; ++r) {
            if (rv[r]) {
                const int64_t o = (int64_t)(y0 + r) * nx + x0;
                vstore<VX>(A.mom_out + o, ar[r]);
                vstore<VX>(A.mom_out + plane + o, ax[r]);
                vstore<VX>(A.mom_out + 2 * plane + o, ay[r]);
            }
        }
        if (on_left || on_right) {
#pragma unroll
            for (int r = 0; r < K; ++r)
                if (rv[r]) A.phi_out[xw * L + y0 + r] = phx[r];
        }
        if (on_bot || on_top) {
#pragma unroll
            for (int v = 0; v < VX; ++v) A.phi_out[yw * L + x0 + v] = phy[v];
        }

        // Residual partials: sum |u_new - u_old|^2, sum |u_new|^2, max |u_new|^2, from the
        // double moments (the old ones re-read rather than kept in registers).
#pragma unroll
        for (int r = 0; r < K; ++r) {
            if (rv[r]) {
                const int64_t o = (int64_t)(y0 + r) * nx + x0;
                double m0[VX], m1[VX], m2[VX];
                vload<VX>(m0, A.mom_in + o);
                vload<VX>(m1, A.mom_in + plane + o);
                vload<VX>(m2, A.mom_in + 2 * plane + o);
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    // one double division per cell: 1 / r0 = r1 / (r0 r1), 1 / r1 = r0 / (r0 r1)
                    // (a few ulp)
                    const double r0 = 1.0 + m0[v], r1 = 1.0 + ar[r][v];
                    const double inv = 1.0 / (r0 * r1);
                    const double i0 = r1 * inv, i1 = r0 * inv;
                    const double ux0 = m1[v] * i0, uy0 = m2[v] * i0;
                    const double ux1 = ax[r][v] * i1, uy1 = ay[r][v] * i1;
                    const double dx = ux1 - ux0, dy = uy1 - uy0;
                    const double u2 = ux1 * ux1 + uy1 * uy1;
                    num += dx * dx + dy * dy;
                    den += u2;
                    umax = fmax(umax, u2);
                }
            }
        }
    }
    num = wave_sum(num);
    den = wave_sum(den);
    umax = wave_max(umax);
    __shared__ double red[WA][WPT][3];
    if (lane == 0) {
        red[wa][wt][0] = num;
        red[wa][wt][1] = den;
        red[wa][wt][2] = umax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0, b = 0, m = 0;
#pragma unroll
        for (int j = 0; j < WA; ++j)
#pragma unroll
            for (int w = 0; w < WPT; ++w) {
                a += red[j][w][0];
                b += red[j][w][1];
                m = fmax(m, red[j][w][2]);
            }
        part[0] = a;
        part[1] = b;
        part[2] = m;
    }
}


// The reduction block of a launch that reduces its predecessor's residual partials inline: one
// extra block, running beside the tiles, sums them (single-wave order) and records the previous
// step.  Nothing waits for it inside the launch.  If that step met a steady solve's criterion,
// the tiles of this launch still compute one more step into the other buffer, which is never
// read: the state of the recorded step stays intact and every later launch is frozen.
template <class T>
__device__ __forceinline__ void reduce_previous(const StepArgs<T>& A) {
    if (threadIdx.x >= 64 || frozen(A.ctrl)) return;
    double num, den, um;
    wave_partials(A.prev_partials, A.prev_nb, num, den, um);
    if (threadIdx.x == 0) record_step(A.ctrl, num, den, um, 1);
}

template <class T, int VX, int K, int LX, int WPB, int WA, int WX, bool NT, int PD, bool PS>
__global__ void __launch_bounds__(64 * WX * WPB * WA) FDLB_WAVES_ATTR step_kernel(const StepArgs<T> A) {
    const int nb = (int)gridDim.x - (A.prev_nb > 0 ? 1 : 0);  // the last block reduces, if any
    if ((int)blockIdx.x == nb) {
        reduce_previous(A);
        return;
    }
    step_body<T, VX, K, LX, WPB, WA, WX, NT, PD, PS>(A, blockIdx.x, nb, A.partials + 3 * blockIdx.x);
}

// Many problems in one launch: block g works on tile map[g].local of problem map[g].inst.
// Each problem's blocks start at a multiple of 8, so the XCD-aware tile order holds per problem.
template <class T, int VX, int K, int LX, int WPB, int WA, int WX, bool NT, int PD, bool PS>
__global__ void __launch_bounds__(64 * WX * WPB * WA) FDLB_WAVES_ATTR batch_step_kernel(const BlockMap* __restrict__ map,
                                                                        const StepArgs<T>* __restrict__ args) {
    const BlockMap m = map[blockIdx.x];
    if (m.inst < 0) return;  // padding block
    const StepArgs<T> A = args[m.inst];
    if (m.local == m.nb) {  // the problem's reduction block
        if (A.prev_nb > 0) reduce_previous(A);
        return;
    }
    step_body<T, VX, K, LX, WPB, WA, WX, NT, PD, PS>(A, m.local, m.nb, A.partials + 3 * m.local);
}

// ---------------------------------------------------------------------------
// Residual: second stage of the reduction, and the step bookkeeping.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void reduce_body(const double* __restrict__ partials, int nblocks,
                                            double* __restrict__ ctrl, int64_t inc) {
    __shared__ double s[3][256];
    double a = 0, b = 0, m = 0;
    for (int i = threadIdx.x; i < nblocks; i += 256) {
        a += partials[3 * i];
        b += partials[3 * i + 1];
        m = fmax(m, partials[3 * i + 2]);
    }
    s[0][threadIdx.x] = a;
    s[1][threadIdx.x] = b;
    s[2][threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s[0][threadIdx.x] += s[0][threadIdx.x + o];
            s[1][threadIdx.x] += s[1][threadIdx.x + o];
            s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) record_step(ctrl, s[0][0], s[1][0], s[2][0], inc);
}

// The closing reduction of a chunk whose steps reduced their predecessors inline: the same
// single-wave order, run by wave 0 of the block.
__device__ __forceinline__ void reduce_wave_body(const double* __restrict__ partials, int nblocks,
                                                 double* __restrict__ ctrl) {
    if (threadIdx.x >= 64) return;
    double num, den, um;
    wave_partials(partials, nblocks, num, den, um);
    if (threadIdx.x == 0) record_step(ctrl, num, den, um, 1);
}

__global__ void __launch_bounds__(256) reduce_kernel(const double* __restrict__ partials, int nblocks,
                                                     double* __restrict__ ctrl, int64_t inc) {
    if (frozen(ctrl)) return;
    reduce_body(partials, nblocks, ctrl, inc);
}

__global__ void __launch_bounds__(64) reduce_wave_kernel(const double* __restrict__ partials, int nblocks,
                                                         double* __restrict__ ctrl) {
    if (frozen(ctrl)) return;
    reduce_wave_body(partials, nblocks, ctrl);
}

// One block per problem of a batch.
__global__ void __launch_bounds__(256) batch_reduce_kernel(const ReduceArgs* __restrict__ ra) {
    const ReduceArgs r = ra[blockIdx.x];
    if (r.nb <= 0 || frozen(r.ctrl)) return;
    if (r.wave_order) reduce_wave_body(r.partials, r.nb, r.ctrl);
    else reduce_body(r.partials, r.nb, r.ctrl, 1);
}

// ---------------------------------------------------------------------------
// Seeding at equilibrium: h_alpha = w_alpha (rho - 1 + xi_alpha . rho u) (Eqs. 3, 5).
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) seed_kernel(T* __restrict__ h, int q, int64_t plane,
                                                   const VelEntry<double>* __restrict__ vel,
                                                   const double* rho, const double* ux, const double* uy,
                                                   const float* frho, const float* fux, const float* fuy,
                                                   const double* mass_scale) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= plane) return;
    double r = 1.0, u = 0.0, w = 0.0;
    if (rho) r = rho[c];
    else if (frho) r = (double)frho[c];
    if (ux) u = ux[c];
    else if (fux) u = (double)fux[c];
    if (uy) w = uy[c];
    else if (fuy) w = (double)fuy[c];
    if (mass_scale) r *= *mass_scale;
    const double jx = r * u, jy = r * w, rh = r - 1.0;
    for (int e = 0; e < q; ++e) {
        const VelEntry<double> v = vel[e];
        h[(int64_t)v.alpha * plane + c] = (T)(v.w * rh + v.wx * jx + v.wy * jy);
    }
}

// Sum of a float array of cells, and the factor that brings it to `cells`.
__global__ void __launch_bounds__(1024) mass_scale_kernel(const float* __restrict__ rho, int64_t cells,
                                                          double* __restrict__ out) {
    __shared__ double s[1024];
    double a = 0;
    for (int64_t i = threadIdx.x; i < cells; i += 1024) a += (double)rho[i];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    // A total that is not positive cannot be renormalised: the scale is then NaN, so the seeded
    // state is NaN and the next steady solve reports divergence at its first step.
    if (threadIdx.x == 0) *out = s[0] > 0.0 ? (double)cells / s[0] : __builtin_nan("");
}

// ---------------------------------------------------------------------------
// Moments and wall fluxes of a state (after seeding or upload), accumulated
// exactly as the step kernel accumulates them for its output: velocity-table
// order, moments in the storage type, wall fluxes in double.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) moments_kernel(const T* __restrict__ h, double* __restrict__ mom,
                                                      double* __restrict__ phi,
                                                      const VelEntry<T>* __restrict__ vel, int q,
                                                      int nx, int ny, int L, const WallConst* wall) {
    const int64_t plane = (int64_t)nx * ny;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= plane) return;
    const int x = (int)(c % nx), y = (int)(c / nx);
    double r = 0, jx = 0, jy = 0;
    double pb = 0, pt = 0, pl = 0, pr = 0;
    for (int e = 0; e < q; ++e) {
        const VelEntry<T> v = vel[e];
        const T f = h[(int64_t)v.alpha * plane + c];
        const double fd = (double)f;
        r += fd;
        jx += (double)v.xx * fd;
        jy += (double)v.xy * fd;
        if (v.xy < 0) pb += -(double)v.xy * (double)f;
        else pt += (double)v.xy * (double)f;
        if (v.xx < 0) pl += -(double)v.xx * (double)f;
        else pr += (double)v.xx * (double)f;
    }
    mom[c] = r;
    mom[plane + c] = jx;
    mom[2 * plane + c] = jy;
    if (wall[BOTTOM].active && y == 0) phi[BOTTOM * L + x] = pb;
    if (wall[TOP].active && y == ny - 1) phi[TOP * L + x] = pt;
    if (wall[LEFT].active && x == 0) phi[LEFT * L + y] = pl;
    if (wall[RIGHT].active && x == nx - 1) phi[RIGHT * L + y] = pr;
}

// ---------------------------------------------------------------------------
// Output fields: rho, u (Eqs. 6-7) and the xy stress of the relaxed state.
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) post_kernel(const T* __restrict__ h,
                                                   const VelEntry<double>* __restrict__ vel, int q,
                                                   int nx, int ny, double omega, double* __restrict__ out) {
    const int64_t plane = (int64_t)nx * ny;
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= plane) return;
    double r = 0, jx = 0, jy = 0;
    for (int e = 0; e < q; ++e) {
        const VelEntry<double> v = vel[e];
        const double f = (double)h[(int64_t)v.alpha * plane + c];
        r += f;
        jx += v.xx * f;
        jy += v.xy * f;
    }
    double pxy = 0;
    for (int e = 0; e < q; ++e) {
        const VelEntry<double> v = vel[e];
        const double f = (double)h[(int64_t)v.alpha * plane + c];
        const double g = (1.0 - omega) * f + omega * (v.w * r + v.wx * jx + v.wy * jy);
        pxy += v.xx * v.xy * g;
    }
    const double rho = 1.0 + r;
    out[c] = rho;
    out[plane + c] = jx / rho;
    out[2 * plane + c] = jy / rho;
    out[3 * plane + c] = pxy;
}

// Face state along a wall: arriving/grazing populations from the wall cell's relaxed
// values, leaving ones from the emission of Eq. (8) with rho_w of Eq. (9).
template <class T>
__global__ void __launch_bounds__(256) wall_profile_kernel(const T* __restrict__ h,
                                                           const VelEntry<double>* __restrict__ vel, int q,
                                                           int nx, int ny, int wall, WallConst wc,
                                                           double omega, double* __restrict__ out) {
    const int64_t plane = (int64_t)nx * ny;
    const int n = (wall == BOTTOM || wall == TOP) ? nx : ny;
    const int pos = blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= n) return;
    int x, y;
    if (wall == BOTTOM) { x = pos; y = 0; }
    else if (wall == TOP) { x = pos; y = ny - 1; }
    else if (wall == LEFT) { x = 0; y = pos; }
    else { x = nx - 1; y = pos; }
    const int64_t c = (int64_t)y * nx + x;
    double r = 0, jx = 0, jy = 0;
    for (int e = 0; e < q; ++e) {
        const VelEntry<double> v = vel[e];
        const double f = (double)h[(int64_t)v.alpha * plane + c];
        r += f;
        jx += v.xx * f;
        jy += v.xy * f;
    }
    auto xn = [&](const VelEntry<double>& v) {
        return wall == BOTTOM ? v.xy : wall == TOP ? -v.xy : wall == LEFT ? v.xx : -v.xx;
    };
    auto xt = [&](const VelEntry<double>& v) { return (wall == BOTTOM || wall == TOP) ? v.xx : v.xy; };
    double s = 0;
    for (int e = 0; e < q; ++e) {
        const VelEntry<double> v = vel[e];
        const double n_ = xn(v);
        if (n_ < 0) {
            const double f = (double)h[(int64_t)v.alpha * plane + c];
            s += -n_ * ((1.0 - omega) * f + omega * (v.w * r + v.wx * jx + v.wy * jy));
        }
    }
    const double P = wc.c0 + wc.k * s;  // rho_w - 1
    double fr = 0, ft = 0, fp = 0;
    for (int e = 0; e < q; ++e) {
        const VelEntry<double> v = vel[e];
        double graw;
        if (xn(v) > 0) {
            graw = v.w * (1.0 + P) * (1.0 + xt(v) * wc.u);
        } else {
            const double f = (double)h[(int64_t)v.alpha * plane + c];
            graw = v.w + (1.0 - omega) * f + omega * (v.w * r + v.wx * jx + v.wy * jy);
        }
        fr += graw;
        ft += xt(v) * graw;
        fp += v.xx * v.xy * graw;
    }
    out[pos] = fr;
    out[n + pos] = ft / fr;
    out[2 * n + pos] = fp;
}

// Raw populations <-> stored deviations, for planes [a0, a1) through a compact buffer.
template <class T>
__global__ void __launch_bounds__(256) to_raw_kernel(const T* __restrict__ h, const double* __restrict__ w_nat,
                                                     int a0, int a1, int64_t plane, double* __restrict__ f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= plane * (a1 - a0)) return;
    const int a = a0 + (int)(i / plane);
    f[i] = w_nat[a] + (double)h[(int64_t)a * plane + i % plane];
}

template <class T>
__global__ void __launch_bounds__(256) from_raw_kernel(const double* __restrict__ f,
                                                       const double* __restrict__ w_nat, int a0, int a1,
                                                       int64_t plane, T* __restrict__ h) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= plane * (a1 - a0)) return;
    const int a = a0 + (int)(i / plane);
    h[(int64_t)a * plane + i % plane] = (T)(f[i] - w_nat[a]);
}

// Float deviations -> double deviations (exact), for the switch of a mixed-precision state.
__global__ void __launch_bounds__(256) widen_kernel(const float* __restrict__ src, double* __restrict__ dst,
                                                    int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (double)src[i];
}

__global__ void __launch_bounds__(256) gather_ctrl_kernel(const double* const* __restrict__ ptrs, int n,
                                                          double* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < 8 * n) out[k] = ptrs[k / 8][k % 8];
}

// Streaming copy for the bandwidth ceiling: each thread keeps 4 x 16-byte loads in flight.  NTL /
// NTS: non-temporal loads / stores (the step kernels load plainly and store non-temporally).
constexpr int COPY_UNROLL = 4;
typedef float copy_vec_t __attribute__((ext_vector_type(4)));
template <bool NTL, bool NTS>
__global__ void __launch_bounds__(256) copy_kernel(copy_vec_t* __restrict__ dst, const copy_vec_t* __restrict__ src,
                                                   int64_t n16) {
    const int64_t chunk = (int64_t)blockDim.x * COPY_UNROLL;
    for (int64_t base = (int64_t)blockIdx.x * chunk; base < n16; base += (int64_t)gridDim.x * chunk) {
        copy_vec_t v[COPY_UNROLL];
#pragma unroll
        for (int u = 0; u < COPY_UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
            if (i < n16) {
                if constexpr (NTL) v[u] = __builtin_nontemporal_load(src + i);
                else v[u] = src[i];
            }
        }
#pragma unroll
        for (int u = 0; u < COPY_UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
            if (i < n16) {
                if constexpr (NTS) __builtin_nontemporal_store(v[u], dst + i);
                else dst[i] = v[u];
            }
        }
    }
}

// Read-only stream (plain loads): every thread sums its 16-byte vectors; one vector per block
// is written (dst must hold gridDim.x vectors), so the loads cannot be dropped.
__global__ void __launch_bounds__(256) read_stream_kernel(copy_vec_t* __restrict__ dst,
                                                          const copy_vec_t* __restrict__ src, int64_t n16) {
    const int64_t chunk = (int64_t)blockDim.x * COPY_UNROLL;
    copy_vec_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int64_t base = (int64_t)blockIdx.x * chunk; base < n16; base += (int64_t)gridDim.x * chunk) {
#pragma unroll
        for (int u = 0; u < COPY_UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
            if (i < n16) acc += src[i];
        }
    }
    __shared__ copy_vec_t s[256];
    s[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        copy_vec_t t = s[0];
        for (int k = 1; k < 256; ++k) t += s[k];
        dst[blockIdx.x] = t;
    }
}

// Write-only stream (non-temporal stores of a constant).
__global__ void __launch_bounds__(256) write_stream_kernel(copy_vec_t* __restrict__ dst, int64_t n16) {
    const int64_t chunk = (int64_t)blockDim.x * COPY_UNROLL;
    const copy_vec_t v = {1.f, 2.f, 3.f, 4.f};
    for (int64_t base = (int64_t)blockIdx.x * chunk; base < n16; base += (int64_t)gridDim.x * chunk) {
#pragma unroll
        for (int u = 0; u < COPY_UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
            if (i < n16) __builtin_nontemporal_store(v, dst + i);
        }
    }
}
__global__ void copy_tail_kernel(char* __restrict__ dst, const char* __restrict__ src, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// Tile shapes and launchers.
// ---------------------------------------------------------------------------
// Compiled tile shapes: id, type, VX, K, LX, WPB, WA, WX, NT, PD (velocity planes prefetched).
#ifndef FDLB_TILES_FP32
#define FDLB_TILES_FP32(X)                \
    X(0, float, 4, 2, 64, 4, 1, 1, 1, 1)  \
    X(1, float, 4, 2, 16, 4, 1, 1, 1, 1)  \
    X(2, float, 4, 2, 32, 4, 1, 1, 1, 1)  \
    X(3, float, 4, 1, 64, 4, 1, 1, 1, 1)  \
    X(4, float, 4, 4, 16, 2, 1, 1, 1, 1)  \
    X(5, float, 2, 4, 64, 4, 1, 1, 1, 1)  \
    X(6, float, 1, 4, 64, 4, 1, 1, 0, 1)  \
    X(7, float, 1, 4, 1, 1, 1, 1, 0, 1)   \
    X(8, float, 1, 2, 16, 1, 1, 1, 0, 1)  \
    X(9, float, 4, 1, 16, 4, 1, 1, 1, 1)  \
    X(10, float, 1, 1, 16, 1, 1, 1, 0, 1) \
    X(11, float, 4, 1, 16, 1, 4, 1, 0, 1) \
    X(12, float, 1, 1, 64, 1, 8, 1, 0, 1) \
    X(13, float, 4, 1, 64, 1, 4, 1, 0, 1) \
    X(14, float, 1, 4, 1, 1, 4, 1, 0, 1)  \
    X(15, float, 2, 1, 32, 1, 8, 1, 0, 1) \
    X(16, float, 4, 1, 16, 2, 2, 1, 0, 1) \
    X(17, float, 4, 2, 64, 1, 1, 4, 1, 1) \
    X(18, float, 4, 1, 64, 1, 1, 4, 1, 1) \
    X(19, float, 4, 2, 64, 2, 1, 2, 1, 1) \
    X(20, float, 4, 4, 64, 1, 1, 4, 1, 1) \
    X(21, float, 1, 1, 32, 1, 8, 1, 0, 1) \
    X(22, float, 2, 1, 64, 1, 8, 1, 0, 1) \
    X(23, float, 4, 2, 16, 1, 4, 1, 0, 1) \
    X(24, float, 2, 1, 32, 1, 4, 1, 0, 1) \
    X(25, float, 4, 2, 16, 1, 8, 1, 0, 1) \
    X(26, float, 1, 1, 1, 1, 8, 1, 0, 1) \
    X(27, float, 1, 2, 1, 1, 4, 1, 0, 1) \
    X(28, float, 4, 2, 16, 1, 4, 1, 1, 1) \
    X(29, float, 4, 1, 16, 1, 4, 1, 1, 1) \
    X(30, float, 4, 2, 16, 1, 2, 1, 1, 1)
#endif

#ifndef FDLB_TILES_FP64
#define FDLB_TILES_FP64(X)                 \
    X(0, double, 2, 2, 64, 4, 1, 1, 1, 1)  \
    X(1, double, 2, 2, 16, 4, 1, 1, 1, 1)  \
    X(2, double, 2, 2, 32, 4, 1, 1, 1, 1)  \
    X(3, double, 1, 2, 64, 4, 1, 1, 0, 1)  \
    X(4, double, 1, 4, 1, 1, 1, 1, 0, 1)   \
    X(5, double, 1, 2, 16, 1, 1, 1, 0, 1)  \
    X(6, double, 2, 1, 64, 4, 1, 1, 1, 1)  \
    X(7, double, 1, 1, 16, 1, 1, 1, 0, 1)  \
    X(8, double, 2, 1, 16, 1, 4, 1, 0, 1)  \
    X(9, double, 1, 1, 64, 1, 8, 1, 0, 1)  \
    X(10, double, 1, 4, 1, 1, 4, 1, 0, 1)  \
    X(11, double, 2, 1, 32, 1, 8, 1, 0, 1) \
    X(12, double, 2, 2, 64, 1, 1, 4, 1, 1) \
    X(13, double, 2, 1, 64, 1, 1, 4, 1, 1) \
    X(14, double, 1, 1, 32, 1, 8, 1, 0, 1) \
    X(15, double, 2, 2, 16, 1, 4, 1, 0, 1) \
    X(16, double, 2, 1, 32, 1, 4, 1, 0, 1) \
    X(17, double, 1, 1, 1, 1, 4, 1, 0, 1)  \
    X(18, double, 1, 2, 1, 1, 4, 1, 0, 1)  \
    X(19, double, 1, 4, 1, 1, 8, 1, 0, 1)  \
    X(20, double, 1, 1, 1, 1, 8, 1, 0, 1)
#endif

const std::vector<TileShape>& tile_shapes(int precision) {
#define FDLB_SHAPE(id, T, VX, K, LX, WPB, WA, WX, NT, PD) TileShape{VX, LX, K, WPB, WA, WX, NT, PD},
    static const std::vector<TileShape> s32 = {FDLB_TILES_FP32(FDLB_SHAPE)};
    static const std::vector<TileShape> s64 = {FDLB_TILES_FP64(FDLB_SHAPE)};
#undef FDLB_SHAPE
    return precision == FDLB_FP32 ? s32 : s64;
}

template <>
void launch_step<float>(int tile, const StepArgs<float>& a, int nblocks, hipStream_t stream) {
    switch (tile) {
#define FDLB_CASE(id, T, VX, K, LX, WPB, WA, WX, NT, PD)                                                         \
    case id:                                                                                                \
        if (a.pseudo)                                                                                       \
            hipLaunchKernelGGL((step_kernel<T, VX, K, LX, WPB, WA, WX, NT, PD, true>), dim3(nblocks),       \
                               dim3(64 * WX * WPB * WA), 0, stream, a);                                     \
        else                                                                                                \
            hipLaunchKernelGGL((step_kernel<T, VX, K, LX, WPB, WA, WX, NT, PD, false>), dim3(nblocks),      \
                               dim3(64 * WX * WPB * WA), 0, stream, a);                                     \
        break;
        FDLB_TILES_FP32(FDLB_CASE)
#undef FDLB_CASE
        default: throw Error(FDLB_EINVAL, "unknown tile shape");
    }
    FDLB_HIP(hipGetLastError());
}

template <>
void launch_step<double>(int tile, const StepArgs<double>& a, int nblocks, hipStream_t stream) {
    switch (tile) {
#define FDLB_CASE(id, T, VX, K, LX, WPB, WA, WX, NT, PD)                                                         \
    case id:                                                                                                \
        if (a.pseudo)                                                                                       \
            hipLaunchKernelGGL((step_kernel<T, VX, K, LX, WPB, WA, WX, NT, PD, true>), dim3(nblocks),       \
                               dim3(64 * WX * WPB * WA), 0, stream, a);                                     \
        else                                                                                                \
            hipLaunchKernelGGL((step_kernel<T, VX, K, LX, WPB, WA, WX, NT, PD, false>), dim3(nblocks),      \
                               dim3(64 * WX * WPB * WA), 0, stream, a);                                     \
        break;
        FDLB_TILES_FP64(FDLB_CASE)
#undef FDLB_CASE
        default: throw Error(FDLB_EINVAL, "unknown tile shape");
    }
    FDLB_HIP(hipGetLastError());
}

template <>
void launch_batch_step<float>(int tile, const BlockMap* map, const StepArgs<float>* args, int nblocks, bool pseudo,
                              hipStream_t stream) {
    switch (tile) {
#define FDLB_CASE(id, T, VX, K, LX, WPB, WA, WX, NT, PD)                                                         \
    case id:                                                                                                \
        if (pseudo)                                                                                         \
            hipLaunchKernelGGL((batch_step_kernel<T, VX, K, LX, WPB, WA, WX, NT, PD, true>), dim3(nblocks), \
                               dim3(64 * WX * WPB * WA), 0, stream, map, args);                             \
        else                                                                                                \
            hipLaunchKernelGGL((batch_step_kernel<T, VX, K, LX, WPB, WA, WX, NT, PD, false>), dim3(nblocks),\
                               dim3(64 * WX * WPB * WA), 0, stream, map, args);                             \
        break;
        FDLB_TILES_FP32(FDLB_CASE)
#undef FDLB_CASE
        default: throw Error(FDLB_EINVAL, "unknown tile shape");
    }
    FDLB_HIP(hipGetLastError());
}

template <>
void launch_batch_step<double>(int tile, const BlockMap* map, const StepArgs<double>* args, int nblocks, bool pseudo,
                              hipStream_t stream) {
    switch (tile) {
#define FDLB_CASE(id, T, VX, K, LX, WPB, WA, WX, NT, PD)                                                         \
    case id:                                                                                                \
        if (pseudo)                                                                                         \
            hipLaunchKernelGGL((batch_step_kernel<T, VX, K, LX, WPB, WA, WX, NT, PD, true>), dim3(nblocks), \
                               dim3(64 * WX * WPB * WA), 0, stream, map, args);                             \
        else                                                                                                \
            hipLaunchKernelGGL((batch_step_kernel<T, VX, K, LX, WPB, WA, WX, NT, PD, false>), dim3(nblocks),\
                               dim3(64 * WX * WPB * WA), 0, stream, map, args);                             \
        break;
        FDLB_TILES_FP64(FDLB_CASE)
#undef FDLB_CASE
        default: throw Error(FDLB_EINVAL, "unknown tile shape");
    }
    FDLB_HIP(hipGetLastError());
}

void launch_batch_reduce(const ReduceArgs* ra, int n, hipStream_t stream) {
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(n), dim3(256), 0, stream, ra);
    FDLB_HIP(hipGetLastError());
}

void launch_reduce_wave(const double* partials, int nblocks, double* ctrl, hipStream_t stream) {
    hipLaunchKernelGGL(reduce_wave_kernel, dim3(1), dim3(64), 0, stream, partials, nblocks, ctrl);
    FDLB_HIP(hipGetLastError());
}

void launch_reduce(const double* partials, int nblocks, double* ctrl, int64_t inc, hipStream_t stream) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, stream, partials, nblocks, ctrl, inc);
    FDLB_HIP(hipGetLastError());
}

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <class T>
void launch_seed(T* h, int q, int64_t plane, const VelEntry<double>* vel, const double* rho,
                 const double* ux, const double* uy, const float* frho, const float* fux, const float* fuy,
                 const double* mass_scale, hipStream_t stream) {
    hipLaunchKernelGGL(seed_kernel<T>, dim3(blocks_for(plane, 256)), dim3(256), 0, stream, h, q, plane, vel,
                       rho, ux, uy, frho, fux, fuy, mass_scale);
    FDLB_HIP(hipGetLastError());
}

void launch_mass_scale(const float* frho, int64_t cells, double* scale_out, hipStream_t stream) {
    hipLaunchKernelGGL(mass_scale_kernel, dim3(1), dim3(1024), 0, stream, frho, cells, scale_out);
    FDLB_HIP(hipGetLastError());
}

template <class T>
void launch_moments(const T* h, double* mom, double* phi, const VelEntry<T>* vel, int q, int nx, int ny,
                    int L, const WallConst* wall, hipStream_t stream) {
    hipLaunchKernelGGL(moments_kernel<T>, dim3(blocks_for((int64_t)nx * ny, 256)), dim3(256), 0, stream, h,
                       mom, phi, vel, q, nx, ny, L, wall);
    FDLB_HIP(hipGetLastError());
}

template <class T>
void launch_post(const T* h, const VelEntry<double>* vel, int q, int nx, int ny, double omega, double* out,
                 hipStream_t stream) {
    hipLaunchKernelGGL(post_kernel<T>, dim3(blocks_for((int64_t)nx * ny, 256)), dim3(256), 0, stream, h, vel,
                       q, nx, ny, omega, out);
    FDLB_HIP(hipGetLastError());
}

template <class T>
void launch_wall_profile(const T* h, const VelEntry<double>* vel, int q, int nx, int ny, int wall,
                         const WallConst* wc, double omega, double* out, hipStream_t stream) {
    const int n = (wall == BOTTOM || wall == TOP) ? nx : ny;
    hipLaunchKernelGGL(wall_profile_kernel<T>, dim3(blocks_for(n, 256)), dim3(256), 0, stream, h, vel, q, nx,
                       ny, wall, *wc, omega, out);
    FDLB_HIP(hipGetLastError());
}

template <class T>
void launch_to_raw(const T* h, const double* w_nat, int a0, int a1, int64_t plane, double* f,
                   hipStream_t stream) {
    hipLaunchKernelGGL(to_raw_kernel<T>, dim3(blocks_for(plane * (a1 - a0), 256)), dim3(256), 0, stream, h,
                       w_nat, a0, a1, plane, f);
    FDLB_HIP(hipGetLastError());
}

template <class T>
void launch_from_raw(const double* f, const double* w_nat, int a0, int a1, int64_t plane, T* h,
                     hipStream_t stream) {
    hipLaunchKernelGGL(from_raw_kernel<T>, dim3(blocks_for(plane * (a1 - a0), 256)), dim3(256), 0, stream, f,
                       w_nat, a0, a1, plane, h);
    FDLB_HIP(hipGetLastError());
}

void launch_widen(const float* src, double* dst, int64_t n, hipStream_t stream) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>(16384, (n + 255) / 256);
    hipLaunchKernelGGL(widen_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, src, dst, n);
    FDLB_HIP(hipGetLastError());
}

void launch_gather_ctrl(const double* const* ptrs, int n, double* out, hipStream_t stream) {
    if (n <= 0) return;
    hipLaunchKernelGGL(gather_ctrl_kernel, dim3((8 * n + 255) / 256), dim3(256), 0, stream, ptrs, n, out);
    FDLB_HIP(hipGetLastError());
}

void launch_copy(void* dst, const void* src, size_t bytes, hipStream_t stream, int mode) {
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 > 0) {
        // 4 loads in flight per thread over 32768 blocks measured fastest on MI355X for multi-GiB
        // copies (5.7 TB/s; 8 per thread or fewer blocks: 5.0-5.5 TB/s).
        const int64_t blocks = std::min<int64_t>(32768, (n16 + 256 * COPY_UNROLL - 1) / (256 * COPY_UNROLL));
        copy_vec_t* d = (copy_vec_t*)dst;
        const copy_vec_t* sv = (const copy_vec_t*)src;
        switch (mode) {
            case FDLB_COPY_PLAIN: hipLaunchKernelGGL((copy_kernel<false, false>), dim3((unsigned)blocks), dim3(256), 0, stream, d, sv, n16); break;
            case FDLB_COPY_NT_LOAD: hipLaunchKernelGGL((copy_kernel<true, false>), dim3((unsigned)blocks), dim3(256), 0, stream, d, sv, n16); break;
            case FDLB_COPY_NT_STORE: hipLaunchKernelGGL((copy_kernel<false, true>), dim3((unsigned)blocks), dim3(256), 0, stream, d, sv, n16); break;
            case FDLB_COPY_NT: hipLaunchKernelGGL((copy_kernel<true, true>), dim3((unsigned)blocks), dim3(256), 0, stream, d, sv, n16); break;
            case FDLB_COPY_READ: hipLaunchKernelGGL(read_stream_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, d, sv, n16); break;
            case FDLB_COPY_WRITE: hipLaunchKernelGGL(write_stream_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, d, n16); break;
            default: throw Error(FDLB_EINVAL, "unknown copy mode");
        }
        FDLB_HIP(hipGetLastError());
    }
    const int64_t tail = (int64_t)bytes - n16 * 16;
    if (tail > 0 && mode <= FDLB_COPY_NT) {
        hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(16), 0, stream, (char*)dst + n16 * 16,
                           (const char*)src + n16 * 16, tail);
        FDLB_HIP(hipGetLastError());
    }
}

#define FDLB_INST(T)                                                                                      \
    template void launch_seed<T>(T*, int, int64_t, const VelEntry<double>*, const double*, const double*, \
                                 const double*, const float*, const float*, const float*, const double*, \
                                 hipStream_t);                                                            \
    template void launch_moments<T>(const T*, double*, double*, const VelEntry<T>*, int, int, int, int,   \
                                    const WallConst*, hipStream_t);                                       \
    template void launch_post<T>(const T*, const VelEntry<double>*, int, int, int, double, double*,       \
                                 hipStream_t);                                                            \
    template void launch_wall_profile<T>(const T*, const VelEntry<double>*, int, int, int, int,           \
                                         const WallConst*, double, double*, hipStream_t);                 \
    template void launch_to_raw<T>(const T*, const double*, int, int, int64_t, double*, hipStream_t);     \
    template void launch_from_raw<T>(const double*, const double*, int, int, int64_t, T*, hipStream_t);
FDLB_INST(float)
FDLB_INST(double)
#undef FDLB_INST

}  // namespace fdlb
