// sphx_runtime.hip -- host runtime of the MI355X Riemann-WCSPH library:
// context, device buffers, HIP-graph capture of the advection step and the
// C ABI declared in include/sphx.h. All particle arithmetic runs in the
// kernels of sphx_device.hpp; the host only sizes buffers, launches,
// captures graphs and marshals arrays in and out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "sphx.h"
#include "sphx_device.hpp"

using namespace sphx;

struct EngineBase;

struct sphx_ctx {
    sphx_params prm;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    std::unique_ptr<EngineBase> eng;
    int fail(int code, const std::string& msg)
    {
        err = msg;
        return code;
    }
};

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return ctx->fail(SPHX_EHIP, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

#define RETCHK(expr)          \
    do {                      \
        int r_ = (expr);      \
        if (r_ != SPHX_OK)    \
            return r_;        \
    } while (0)

struct EngineBase {
    virtual ~EngineBase() {}
    virtual int init() = 0;
    virtual int set_fluid(int64_t n, const double* pos, const double* vel, const double* rho, const double* drho) = 0;
    virtual int set_walls(int64_t n, const double* pos, const double* nrm) = 0;
    virtual int build_neighbors() = 0;
    virtual int get_neighbors(int kind, int64_t* off, int64_t* idx, int64_t cap, int64_t* n_out) = 0;
    virtual int density_reinit() = 0;
    virtual int time_steps(double* dt_ad, double* dt_ac) = 0;
    virtual int compute_rates(double dt, double* dvdt, double* drhodt) = 0;
    virtual int advance(int32_t n_steps, double t_stop, int64_t* nsub, double* t_out) = 0;
    virtual int get_field(int which, double* out) = 0;
    virtual int diagnostics(sphx_diag* out) = 0;
    virtual int profile(int32_t reps, double* ms) = 0;
    virtual int counts(int64_t* out) = 0;
};

static inline int nblk(long long n) { return (int)((n + BLOCK - 1) / BLOCK); }

template <int D, typename real>
struct Engine final : EngineBase {
    using G = typename GeoSel<D, real>::T;
    sphx_ctx* ctx;
    hipStream_t s;
    KP<real> P{};
    static constexpr int LN = D == 2 ? 4 : 8;   // lanes per particle in the pair kernels
    static constexpr int LB = 4;  // lanes per particle in the neighbour build (measured best of 1-64)
    int ncell = 0, nsub_q = 5, steps_per_graph = 2;
    int maxn = 0, maxw = 0;
    // fluid: two state sets (current and gather target)
    int nf = 0, cap = 0;
    double* x[2][3] = {};
    R4<real>* st[2] = {};
    real* dr3[2] = {};
    G* geo[2] = {};
    int32_t* id[2] = {};
    int32_t* cell[2] = {};
    R4<real>* hf = nullptr;
    uint32_t* nbr = nullptr;
    int32_t* ncnt = nullptr;
    uint32_t* wnb = nullptr;
    int32_t* wcnt = nullptr;
    int32_t *key = nullptr, *rank = nullptr, *perm = nullptr;
    int32_t *cnt = nullptr, *fstart = nullptr, *bsum = nullptr;
    real* acc_out = nullptr;
    real* drho_out = nullptr;
    unsigned long long* vslot = nullptr;  // |v| maxima slots of the density relaxation (zero between uses)
    double* outbuf = nullptr;
    double* stage = nullptr;
    size_t stage_n = 0;
    double* diag_part = nullptr;
    double* diag_out = nullptr;
    // state backup for calls that must leave the state unchanged
    R4<real>* bk_st = nullptr;
    real* bk_dr = nullptr;
    double* bk_x[3] = {};
    // walls
    int nw = 0, wcap = 0;
    double* wx[3] = {};
    G* wgeo = nullptr;
    G* wnrm = nullptr;
    int32_t* wid = nullptr;
    int32_t* wstart = nullptr;
    // control
    Ctrl* ctrl = nullptr;
    Ctrl* hctrl = nullptr;  // pinned mirror
    int cur = 0;
    long long cur_steps = 0;
    bool configured = false;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // steps_per_graph steps, by start parity
    hipGraphExec_t gone[2] = {nullptr, nullptr};    // one step, by start parity
    std::vector<void*> fluid_allocs, wall_allocs;

    explicit Engine(sphx_ctx* c) : ctx(c), s(c->stream) {}

    ~Engine() override
    {
        drop_graphs();
        free_list(fluid_allocs);
        free_list(wall_allocs);
        (void)hipFree(ctrl);
        (void)hipFree(cnt);
        (void)hipFree(fstart);
        (void)hipFree(bsum);
        (void)hipFree(wstart);
        (void)hipFree(diag_out);
        if (hctrl) (void)hipHostFree(hctrl);
    }

    static void free_list(std::vector<void*>& v)
    {
        for (void* p : v) (void)hipFree(p);
        v.clear();
    }

    void drop_graphs()
    {
        for (hipGraphExec_t* g : {&gexec[0], &gexec[1], &gone[0], &gone[1]})
            if (*g) {
                (void)hipGraphExecDestroy(*g);
                *g = nullptr;
            }
    }

    template <typename T>
    int dalloc(std::vector<void*>& list, T*& p, size_t count)
    {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
        if (e != hipSuccess) return ctx->fail(SPHX_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        list.push_back(q);
        p = (T*)q;
        return SPHX_OK;
    }

    // ------------------------------------------------------------------
    int init() override
    {
        const sphx_params& q = ctx->prm;
        const double PI = 3.14159265358979323846;
        double alpha = D == 2 ? 7.0 / (4.0 * PI) : 21.0 / (16.0 * PI);
        double h = q.h;
        P.rho0 = (real)q.rho0;
        P.rho0d = q.rho0;
        P.c = (real)q.c0;
        P.c0d = q.c0;
        P.c2 = (real)(q.c0 * q.c0);
        P.inv_c2 = (real)(1.0 / (q.c0 * q.c0));
        P.half_inv_c = (real)(0.5 / q.c0);
        double vol = std::pow(q.dp, D);
        P.md = q.rho0 * vol;
        P.m = (real)P.md;
        P.two_m = (real)(2.0 * P.md);
        P.vw = (real)vol;
        P.two_vw = (real)(2.0 * vol);
        P.inv_h = (real)(1.0 / h);
        P.Wc = (real)(alpha / std::pow(h, D));
        P.dWc = (real)(-5.0 * alpha / std::pow(h, D + 1));
        for (int k = 0; k < 3; ++k) P.g[k] = (real)(k < D ? q.gravity[k] : 0.0);
        double rc = 2.0 * h;
        ncell = 1;
        for (int k = 0; k < 3; ++k) {
            if (k < D) {
                double len = q.hi[k] - q.lo[k];
                if (!(len > 0)) return ctx->fail(SPHX_EINVAL, "empty domain box");
                long long n = (long long)std::floor(len / rc);
                while (n > 1 && len / (double)n < rc) --n;
                if (n < 1) n = 1;
                if (n > 100000) return ctx->fail(SPHX_EINVAL, "cell grid too large");
                if (q.periodic[k] && n < 3)
                    return ctx->fail(SPHX_EINVAL, "a periodic axis needs at least 3 cells of size 2h");
                P.n[k] = (int)n;
                P.Ld[k] = len / (double)n;
                P.lo[k] = q.lo[k];
                P.hi[k] = q.hi[k];
                P.period[k] = len;
                P.half_period[k] = 0.5 * len;
                P.periodic[k] = q.periodic[k] ? 1 : 0;
            } else {
                P.n[k] = 1;
                P.Ld[k] = 1.0;
                P.lo[k] = 0.0;
                P.hi[k] = 1.0;
                P.period[k] = 1.0;
                P.half_period[k] = 0.5;
                P.periodic[k] = 0;
            }
            P.L[k] = (real)P.Ld[k];
            ncell *= P.n[k];
        }
        if ((long long)P.n[0] * P.n[1] * P.n[2] > 50000000LL) return ctx->fail(SPHX_EINVAL, "cell grid too large");
        P.rc2 = (2.0 * h) * (2.0 * h);
        if (q.sigma0 > 0) {
            P.sigma0 = q.sigma0;
        } else {
            // lattice sum of W over the dp lattice, self included
            int K = (int)std::ceil(2.0 * h / q.dp) + 1;
            double sum = 0.0;
            for (int a = -K; a <= K; ++a)
                for (int b = -K; b <= K; ++b)
                    for (int c = (D == 3 ? -K : 0); c <= (D == 3 ? K : 0); ++c) {
                        double r = q.dp * std::sqrt((double)(a * a + b * b + c * c));
                        double qq = r / h;
                        if (qq < 2.0) {
                            double sq = 1.0 - 0.5 * qq;
                            sum += alpha / std::pow(h, D) * sq * sq * sq * sq * (1.0 + 2.0 * qq);
                        }
                    }
            P.sigma0 = sum;
        }
        P.cfl_ad_h = q.cfl_ad * h;
        P.cfl_ac_h = q.cfl_ac * h;
        P.u_ref = q.u_ref;
        maxn = D == 2 ? 48 : 128;
        maxw = D == 2 ? 32 : 96;
        P.maxn = maxn;
        P.maxw = maxw;
        nsub_q = q.nsub_queue > 0 ? q.nsub_queue : 5;
        if (nsub_q > 64) nsub_q = 64;
        HIPCHK(hipMalloc((void**)&ctrl, sizeof(Ctrl)));
        HIPCHK(hipHostMalloc((void**)&hctrl, sizeof(Ctrl), hipHostMallocDefault));
        std::memset(hctrl, 0, sizeof(Ctrl));
        HIPCHK(hipMemcpyAsync(ctrl, hctrl, sizeof(Ctrl), hipMemcpyHostToDevice, s));
        HIPCHK(hipMalloc((void**)&cnt, sizeof(int32_t) * (size_t)ncell));
        HIPCHK(hipMalloc((void**)&fstart, sizeof(int32_t) * ((size_t)ncell + 1)));
        HIPCHK(hipMalloc((void**)&wstart, sizeof(int32_t) * ((size_t)ncell + 1)));
        HIPCHK(hipMalloc((void**)&bsum, sizeof(int32_t) * ((size_t)nblk_scan() + 1)));
        HIPCHK(hipMalloc((void**)&diag_out, sizeof(double) * NDIAG));
        HIPCHK(hipMemsetAsync(wstart, 0, sizeof(int32_t) * ((size_t)ncell + 1), s));
        HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)ncell, s));
        HIPCHK(hipStreamSynchronize(s));
        P.nf = 0;
        P.nw = 0;
        return SPHX_OK;
    }

    int nblk_scan() const { return (ncell + SCAN_TILE - 1) / SCAN_TILE; }

    int sync_ctrl()
    {
        HIPCHK(hipMemcpyAsync(hctrl, ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (hctrl->err_pending) {  // raised outside a finalising launch (rates, profiling)
            hctrl->err |= hctrl->err_pending;
            hctrl->err_pending = 0;
            RETCHK(push_ctrl());
            HIPCHK(hipStreamSynchronize(s));
        }
        return SPHX_OK;
    }

    int push_ctrl()
    {
        HIPCHK(hipMemcpyAsync(ctrl, hctrl, sizeof(Ctrl), hipMemcpyHostToDevice, s));
        return SPHX_OK;
    }

    int err_code(uint32_t e)
    {
        if (e & ERR_NAN) return ctx->fail(SPHX_ENAN, "NaN in the particle state");
        if (e & ERR_ESCAPE) return ctx->fail(SPHX_EESCAPE, "a fluid particle left the domain box");
        if (e & ERR_NBR_OVERFLOW) return ctx->fail(SPHX_EOVERFLOW, "neighbour list capacity exceeded");
        return SPHX_OK;
    }

    // ------------------------------------------------------------------
    int alloc_fluid(int n)
    {
        drop_graphs();
        free_list(fluid_allocs);
        cap = n;
        auto& L = fluid_allocs;
        for (int a = 0; a < 2; ++a) {
            for (int k = 0; k < D; ++k) RETCHK(dalloc(L, x[a][k], n));
            if (D == 2) x[a][2] = x[a][1];  // never dereferenced in 2D
            RETCHK(dalloc(L, st[a], n));
            if (D == 3) RETCHK(dalloc(L, dr3[a], n));
            else dr3[a] = nullptr;
            RETCHK(dalloc(L, geo[a], n));
            RETCHK(dalloc(L, id[a], n));
            RETCHK(dalloc(L, cell[a], n));
        }
        RETCHK(dalloc(L, hf, n));
        size_t ncap = (size_t)(n + 63) / 64 * 64;  // whole wave tiles
        RETCHK(dalloc(L, nbr, (size_t)maxn * ncap));
        RETCHK(dalloc(L, ncnt, n));
        RETCHK(dalloc(L, wnb, (size_t)maxw * ncap));
        RETCHK(dalloc(L, wcnt, n));
        RETCHK(dalloc(L, key, n));
        RETCHK(dalloc(L, rank, n));
        RETCHK(dalloc(L, perm, n));
        RETCHK(dalloc(L, acc_out, (size_t)n * D));
        RETCHK(dalloc(L, vslot, 2 * VSLOTS));
        HIPCHK(hipMemsetAsync(vslot, 0, sizeof(unsigned long long) * 2 * VSLOTS, s));
        RETCHK(dalloc(L, drho_out, n));
        RETCHK(dalloc(L, outbuf, (size_t)n * D));
        RETCHK(dalloc(L, diag_part, (size_t)nblk(n) * NDIAG));
        RETCHK(dalloc(L, bk_st, n));
        if (D == 3) RETCHK(dalloc(L, bk_dr, n));
        for (int k = 0; k < D; ++k) RETCHK(dalloc(L, bk_x[k], n));
        if (D == 2) bk_x[2] = bk_x[1];
        return SPHX_OK;
    }

    int ensure_stage(size_t ndoubles)
    {
        if (ndoubles <= stage_n) return SPHX_OK;
        if (stage) {
            (void)hipFree(stage);
            stage = nullptr;
        }
        HIPCHK(hipMalloc((void**)&stage, ndoubles * sizeof(double)));
        stage_n = ndoubles;
        return SPHX_OK;
    }

    int set_fluid(int64_t n, const double* pos, const double* vel, const double* rho, const double* drho) override
    {
        if (n < 0 || (n > 0 && !pos) || n > (int64_t)NBR_MASK) return ctx->fail(SPHX_EINVAL, "bad fluid particle count or positions");
        HIPCHK(hipStreamSynchronize(s));
        if ((int)n > cap || n == 0) RETCHK(alloc_fluid((int)std::max<int64_t>(n, 1)));
        drop_graphs();
        nf = (int)n;
        P.nf = nf;
        P.cap = cap;
        configured = false;
        cur = 0;
        // stage: pos | vel | rho | drho
        size_t nn = (size_t)n;
        RETCHK(ensure_stage(nn * (2 * D + 2)));
        double* dpos = stage;
        double* dvel = stage + nn * D;
        double* drh = stage + nn * 2 * D;
        double* ddr = drh + nn;
        if (n > 0) {
            HIPCHK(hipMemcpyAsync(dpos, pos, nn * D * sizeof(double), hipMemcpyHostToDevice, s));
            if (vel) HIPCHK(hipMemcpyAsync(dvel, vel, nn * D * sizeof(double), hipMemcpyHostToDevice, s));
            if (rho) HIPCHK(hipMemcpyAsync(drh, rho, nn * sizeof(double), hipMemcpyHostToDevice, s));
            if (drho) HIPCHK(hipMemcpyAsync(ddr, drho, nn * sizeof(double), hipMemcpyHostToDevice, s));
            k_load_fluid<D, real><<<nblk(n), BLOCK, 0, s>>>(P, dpos, vel ? dvel : nullptr, rho ? drh : nullptr,
                                                             drho ? ddr : nullptr, x[0][0], x[0][1], x[0][2], st[0],
                                                             dr3[0], id[0]);
            HIPCHK(hipGetLastError());
        }
        std::memset(hctrl, 0, sizeof(Ctrl));
        RETCHK(push_ctrl());
        HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)ncell, s));  // after a failed rebuild
        cur_steps = 0;
        if (n > 0) {
            k_vmax<D, real><<<nblk(n), BLOCK, 0, s>>>(P, ctrl, st[0]);
            k_vmax_fin<real><<<1, 1, 0, s>>>(ctrl);
            HIPCHK(hipGetLastError());
        }
        RETCHK(sync_ctrl());
        return SPHX_OK;
    }

    int set_walls(int64_t n, const double* pos, const double* nrm) override
    {
        if (n < 0 || (n > 0 && (!pos || !nrm)) || n > (int64_t)NBR_MASK) return ctx->fail(SPHX_EINVAL, "bad wall particle count or arrays");
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < D; ++k) {
                double v = pos[i * D + k];
                if (!(v >= P.lo[k] && v < P.hi[k])) return ctx->fail(SPHX_EINVAL, "wall particle outside the domain box");
            }
        HIPCHK(hipStreamSynchronize(s));
        drop_graphs();
        configured = false;
        free_list(wall_allocs);
        nw = (int)n;
        wcap = (int)std::max<int64_t>(n, 1);
        auto& L = wall_allocs;
        for (int k = 0; k < D; ++k) RETCHK(dalloc(L, wx[k], wcap));
        if (D == 2) wx[2] = wx[1];
        RETCHK(dalloc(L, wgeo, wcap));
        RETCHK(dalloc(L, wnrm, wcap));
        RETCHK(dalloc(L, wid, wcap));
        int32_t *wkey, *wrank, *wperm;
        RETCHK(dalloc(L, wkey, wcap));
        RETCHK(dalloc(L, wrank, wcap));
        RETCHK(dalloc(L, wperm, wcap));
        P.nw = nw;
        if (n == 0) {
            HIPCHK(hipMemsetAsync(wstart, 0, sizeof(int32_t) * ((size_t)ncell + 1), s));
            HIPCHK(hipStreamSynchronize(s));
            return SPHX_OK;
        }
        // stage SoA positions and normals (original order)
        size_t nn = (size_t)n;
        RETCHK(ensure_stage(nn * 6));
        std::vector<double> soa(nn * 6, 0.0);
        for (size_t i = 0; i < nn; ++i)
            for (int k = 0; k < D; ++k) {
                soa[k * nn + i] = pos[i * D + k];
                soa[(3 + k) * nn + i] = nrm[i * D + k];
            }
        HIPCHK(hipMemcpyAsync(stage, soa.data(), nn * 6 * sizeof(double), hipMemcpyHostToDevice, s));
        double* sx[3] = {stage, stage + nn, stage + 2 * nn};
        double* sn[3] = {stage + 3 * nn, stage + 4 * nn, stage + 5 * nn};
        HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)ncell, s));
        k_bin<D, real><<<nblk(n), BLOCK, 0, s>>>(P, ctrl, 0, (int)n, sx[0], sx[1], sx[2], wkey, wrank, cnt, 0);
        RETCHK(enqueue_scan(0, wstart));
        k_scatter<<<nblk(n), BLOCK, 0, s>>>(ctrl, 0, (int)n, wkey, wrank, wstart, wperm);
        k_cell_order<<<nblk(ncell), BLOCK, 0, s>>>(ctrl, 0, ncell, wstart, wperm);
        k_gather_wall<D, real><<<nblk(n), BLOCK, 0, s>>>(P, (int)n, wperm, wkey, sx[0], sx[1], sx[2], sn[0], sn[1],
                                                          sn[2], wx[0], wx[1], wx[2], wgeo, wnrm, wid);
        HIPCHK(hipGetLastError());
        RETCHK(sync_ctrl());
        return SPHX_OK;
    }

    int enqueue_scan(int gate, int32_t* out)
    {
        int nb = nblk_scan();
        k_scan_tiles<<<nb, BLOCK, 0, s>>>(ctrl, gate, cnt, out, bsum, ncell);
        k_scan_top<<<1, BLOCK, 0, s>>>(ctrl, gate, bsum, nb);
        k_scan_add<<<nb, BLOCK, 0, s>>>(ctrl, gate, out, bsum, ncell, nb);
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    // S1-S3 from state set a into set b. The cell counters are zero on entry
    // (zeroed at allocation and by every scan that consumes them).
    int enqueue_rebuild(int gate, int a)
    {
        int b = 1 - a;
        k_bin<D, real><<<nblk(nf), BLOCK, 0, s>>>(P, ctrl, gate, nf, x[a][0], x[a][1], x[a][2], key, rank, cnt, 1);
        RETCHK(enqueue_scan(gate, fstart));
        k_scatter<<<nblk(nf), BLOCK, 0, s>>>(ctrl, gate, nf, key, rank, fstart, perm);
        k_place_fluid<D, real><<<nblk(nf), BLOCK, 0, s>>>(P, ctrl, gate, nf, perm, key, fstart, x[a][0], x[a][1],
                                                           x[a][2], st[a], dr3[a], id[a], x[b][0], x[b][1], x[b][2],
                                                           st[b], dr3[b], id[b], cell[b], geo[b]);
        k_neighbors<D, real, LN, LB><<<nblk((long long)nf * LB), BLOCK, 0, s>>>(
            P, ctrl, gate, x[b][0], x[b][1], x[b][2], cell[b], fstart, geo[b], wx[0], wx[1], wx[2], wstart, wgeo, nbr,
            ncnt, wnb, wcnt);
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    // Pressure and density relaxation of sub-step q on set a; `adv`: close
    // sub-step q - 1 first (inside the pressure relaxation).
    int enqueue_substep(int a, int q, int adv, int finalize, real* acc, real* dro)
    {
        k_pressure<D, real, LN><<<nblk((long long)nf * LN), BLOCK, 0, s>>>(P, ctrl, geo[a], wgeo, wnrm, nbr, ncnt, wnb,
                                                                          wcnt, st[a], dr3[a], hf, acc, q, adv, vslot);
        k_density<D, real, LN><<<nblk((long long)nf * LN), BLOCK, 0, s>>>(P, ctrl, finalize, geo[a], wgeo, wnrm, nbr,
                                                                         ncnt, wnb, wcnt, hf, st[a], dr3[a], x[a][0],
                                                                         x[a][1], x[a][2], dro, vslot, q);
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    // One advection step on set a (graph body): re-init, the queued
    // sub-steps, the step end (which prepares the next step), the rebuild.
    int enqueue_step(int a)
    {
        k_reinit<D, real, LN><<<nblk((long long)nf * LN), BLOCK, 0, s>>>(P, ctrl, 1, geo[a], wgeo, nbr, ncnt, wnb, wcnt,
                                                                        st[a]);
        for (int q = 0; q < nsub_q; ++q) RETCHK(enqueue_substep(a, q, q > 0, 1, nullptr, nullptr));
        k_step_end<real><<<1, 64, 0, s>>>(P, ctrl, vslot, nsub_q - 1, 1, 1);
        RETCHK(enqueue_rebuild(1, a));
        return SPHX_OK;
    }

    int capture_one(hipGraphExec_t* out, int parity, int nsteps)
    {
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int rc = SPHX_OK;
        for (int q = 0; q < nsteps && rc == SPHX_OK; ++q) rc = enqueue_step((parity + q) & 1);
        hipError_t e = hipStreamEndCapture(s, &g);
        if (rc != SPHX_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return ctx->fail(SPHX_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            *out = nullptr;
            return ctx->fail(SPHX_EHIP, std::string("graph instantiate failed: ") + hipGetErrorString(e));
        }
        return SPHX_OK;
    }

    int capture_graphs()
    {
        for (int p = 0; p < 2; ++p) {
            if (!gexec[p]) RETCHK(capture_one(&gexec[p], p, steps_per_graph));
            if (!gone[p]) RETCHK(capture_one(&gone[p], p, 1));
        }
        return SPHX_OK;
    }

    // ------------------------------------------------------------------
    int build_neighbors() override
    {
        if (nf == 0) return ctx->fail(SPHX_ESTATE, "no fluid particles");
        RETCHK(sync_ctrl());
        hctrl->err = 0;
        RETCHK(push_ctrl());
        HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)ncell, s));  // a failed rebuild may leave counts
        RETCHK(enqueue_rebuild(0, cur));
        RETCHK(sync_ctrl());
        cur ^= 1;
        if (hctrl->err) {
            configured = false;
            uint32_t e = hctrl->err;
            hctrl->err = 0;
            RETCHK(push_ctrl());
            return err_code(e);
        }
        configured = true;
        return SPHX_OK;
    }

    int get_neighbors(int kind, int64_t* off, int64_t* idx, int64_t cap_idx, int64_t* n_out) override
    {
        if (!configured) return ctx->fail(SPHX_ESTATE, "no neighbour configuration");
        int mx = kind == SPHX_INNER ? maxn : maxw;
        std::vector<int32_t> cnts(nf), ids(nf), oid(std::max(nw, 1));
        size_t ncap = (size_t)(cap + 63) / 64 * 64;
        std::vector<uint32_t> ell((size_t)mx * ncap);
        HIPCHK(hipMemcpyAsync(cnts.data(), kind == SPHX_INNER ? ncnt : wcnt, sizeof(int32_t) * nf, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(ids.data(), id[cur], sizeof(int32_t) * nf, hipMemcpyDeviceToHost, s));
        if (kind != SPHX_INNER && nw > 0)
            HIPCHK(hipMemcpyAsync(oid.data(), wid, sizeof(int32_t) * nw, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(ell.data(), kind == SPHX_INNER ? nbr : wnb, sizeof(uint32_t) * (size_t)mx * ncap,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<int64_t> rowlen(nf + 1, 0);
        for (int i = 0; i < nf; ++i) rowlen[ids[i] + 1] = cnts[i];
        for (int i = 0; i < nf; ++i) rowlen[i + 1] += rowlen[i];
        int64_t total = rowlen[nf];
        if (n_out) *n_out = total;
        if (off)
            for (int i = 0; i <= nf; ++i) off[i] = rowlen[i];
        if (idx) {
            if (cap_idx < total) return ctx->fail(SPHX_ECAP, "neighbour index buffer too small");
            for (int i = 0; i < nf; ++i) {
                int64_t o = rowlen[ids[i]];
                for (int k = 0; k < cnts[i]; ++k) {
                    uint32_t j = ell[ell_at<LN>(i, k, mx)] & NBR_MASK;
                    idx[o + k] = kind == SPHX_INNER ? ids[j] : oid[j];
                }
                std::sort(idx + o, idx + o + cnts[i]);
            }
        }
        return SPHX_OK;
    }

    int density_reinit() override
    {
        if (!configured) return ctx->fail(SPHX_ESTATE, "no neighbour configuration");
        k_reinit<D, real, LN><<<nblk((long long)nf * LN), BLOCK, 0, s>>>(P, ctrl, 0, geo[cur], wgeo, nbr, ncnt, wnb, wcnt, st[cur]);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(s));
        return SPHX_OK;
    }

    int refresh_vmax()
    {
        if (nf > 0) {
            k_vmax<D, real><<<nblk(nf), BLOCK, 0, s>>>(P, ctrl, st[cur]);
            k_vmax_fin<real><<<1, 1, 0, s>>>(ctrl);
            HIPCHK(hipGetLastError());
        }
        return sync_ctrl();
    }

    int time_steps(double* dt_ad, double* dt_ac) override
    {
        if (nf == 0) return ctx->fail(SPHX_ESTATE, "no fluid particles");
        RETCHK(refresh_vmax());
        double vmax = hctrl->vmax;
        if (dt_ad) *dt_ad = P.cfl_ad_h / std::fmax(vmax, P.u_ref);
        if (dt_ac) *dt_ac = P.cfl_ac_h / (P.c0d + vmax);
        return SPHX_OK;
    }

    int backup_state()
    {
        HIPCHK(hipMemcpyAsync(bk_st, st[cur], sizeof(R4<real>) * nf, hipMemcpyDeviceToDevice, s));
        if (D == 3) HIPCHK(hipMemcpyAsync(bk_dr, dr3[cur], sizeof(real) * nf, hipMemcpyDeviceToDevice, s));
        for (int k = 0; k < D; ++k)
            HIPCHK(hipMemcpyAsync(bk_x[k], x[cur][k], sizeof(double) * nf, hipMemcpyDeviceToDevice, s));
        return SPHX_OK;
    }

    int restore_state(const Ctrl& saved)
    {
        HIPCHK(hipMemcpyAsync(st[cur], bk_st, sizeof(R4<real>) * nf, hipMemcpyDeviceToDevice, s));
        if (D == 3) HIPCHK(hipMemcpyAsync(dr3[cur], bk_dr, sizeof(real) * nf, hipMemcpyDeviceToDevice, s));
        for (int k = 0; k < D; ++k)
            HIPCHK(hipMemcpyAsync(x[cur][k], bk_x[k], sizeof(double) * nf, hipMemcpyDeviceToDevice, s));
        *hctrl = saved;
        RETCHK(push_ctrl());
        HIPCHK(hipStreamSynchronize(s));
        return SPHX_OK;
    }

    int compute_rates(double dt, double* dvdt, double* drhodt) override
    {
        if (!configured) return ctx->fail(SPHX_ESTATE, "no neighbour configuration");
        RETCHK(sync_ctrl());
        Ctrl saved = *hctrl;
        RETCHK(backup_state());
        hctrl->ss[0] = SubState{0.0, dt, 0, 1, 0, 0};
        hctrl->err = 0;
        RETCHK(push_ctrl());
        RETCHK(enqueue_substep(cur, 0, 0, 0, acc_out, drho_out));
        if (dvdt) {
            k_unsort_vec<real><<<nblk(nf), BLOCK, 0, s>>>(nf, D, id[cur], acc_out, outbuf);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(dvdt, outbuf, sizeof(double) * (size_t)nf * D, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        if (drhodt) {
            k_unsort_vec<real><<<nblk(nf), BLOCK, 0, s>>>(nf, 1, id[cur], drho_out, outbuf);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(drhodt, outbuf, sizeof(double) * (size_t)nf, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        RETCHK(sync_ctrl());
        uint32_t e = hctrl->err;
        RETCHK(restore_state(saved));
        return err_code(e);
    }

    // Finish an advection step that ran out of queued sub-steps, from the
    // host, one sub-step per synchronisation; then rebuild its configuration
    // and prepare the next step.
    int finish_stalled_step()
    {
        hctrl->err &= ~ERR_STALL;
        RETCHK(push_ctrl());
        int q = nsub_q;
        for (int it = 0; it < 100000; ++it, ++q) {
            RETCHK(enqueue_substep(cur, q, 0, 1, nullptr, nullptr));
            k_step_end<real><<<1, 64, 0, s>>>(P, ctrl, vslot, q, 0, 0);
            HIPCHK(hipGetLastError());
            RETCHK(sync_ctrl());
            if (hctrl->err) return err_code(hctrl->err);
            if (hctrl->rebuild) break;
        }
        if (!hctrl->rebuild) return ctx->fail(SPHX_ESTATE, "advection step did not finish");
        RETCHK(enqueue_rebuild(1, cur));
        k_adv_begin<real><<<1, 1, 0, s>>>(P, ctrl);
        HIPCHK(hipGetLastError());
        RETCHK(sync_ctrl());
        cur ^= 1;
        cur_steps = hctrl->steps_done;
        return err_code(hctrl->err);
    }

    int advance(int32_t n_steps, double t_stop, int64_t* nsub_out, double* t_out) override
    {
        if (nf == 0) return ctx->fail(SPHX_ESTATE, "no fluid particles");
        if (!configured) RETCHK(build_neighbors());
        RETCHK(capture_graphs());
        RETCHK(sync_ctrl());
        long long sub0 = hctrl->nsub_total;
        long long start = hctrl->steps_done;
        cur_steps = start;
        HIPCHK(hipMemcpyAsync(&ctrl->t_stop, &t_stop, sizeof(double), hipMemcpyHostToDevice, s));
        k_adv_begin<real><<<1, 1, 0, s>>>(P, ctrl);
        HIPCHK(hipGetLastError());
        RETCHK(sync_ctrl());
        long long remaining = n_steps;
        while (remaining > 0 && hctrl->t < t_stop) {
            // up to 64 steps per batch, one host synchronisation per batch
            long long batch = std::min<long long>(remaining, 64);
            int pp = cur;
            long long q = 0;
            for (; q + steps_per_graph <= batch; q += steps_per_graph) {
                HIPCHK(hipGraphLaunch(gexec[pp], s));
                pp = (pp + steps_per_graph) & 1;
            }
            for (; q < batch; ++q) {
                HIPCHK(hipGraphLaunch(gone[pp], s));
                pp ^= 1;
            }
            int cur_before = cur;
            long long steps_before = cur_steps;
            RETCHK(sync_ctrl());
            long long done = hctrl->steps_done - steps_before;
            cur = (int)((cur_before + done) & 1);
            cur_steps = hctrl->steps_done;
            if (hctrl->err & ~ERR_STALL) {
                // a NaN or an escape stops the rebuild of the step it occurs in
                if ((hctrl->err & (ERR_ESCAPE | ERR_NAN)) && done > 0) cur = (int)((cur_before + done - 1) & 1);
                configured = false;
                return err_code(hctrl->err);
            }
            if (hctrl->err & ERR_STALL) RETCHK(finish_stalled_step());
            remaining = n_steps - (cur_steps - start);
        }
        if (nsub_out) *nsub_out = hctrl->nsub_total - sub0;
        if (t_out) *t_out = hctrl->t;
        return SPHX_OK;
    }

    int get_field(int which, double* out) override
    {
        if (which < 0 || which > 4 || !out) return ctx->fail(SPHX_EINVAL, "bad field");
        if (nf == 0) return SPHX_OK;
        k_unsort_field<D, real><<<nblk(nf), BLOCK, 0, s>>>(P, which, id[cur], x[cur][0], x[cur][1], x[cur][2], st[cur],
                                                            dr3[cur], outbuf);
        HIPCHK(hipGetLastError());
        size_t cnt_out = (which <= 1 ? (size_t)D : 1) * nf;
        HIPCHK(hipMemcpyAsync(out, outbuf, sizeof(double) * cnt_out, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return SPHX_OK;
    }

    int diagnostics(sphx_diag* out) override
    {
        if (!out) return ctx->fail(SPHX_EINVAL, "NULL output");
        double r[NDIAG] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (nf > 0) {
            k_diag<D, real><<<nblk(nf), BLOCK, 0, s>>>(P, x[cur][0], x[cur][1], x[cur][2], st[cur], diag_part);
            k_diag_fin<<<1, BLOCK, 0, s>>>(diag_part, nblk(nf), diag_out);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(r, diag_out, sizeof(r), hipMemcpyDeviceToHost, s));
        }
        RETCHK(sync_ctrl());
        out->mass = P.md * nf;
        out->momentum[0] = r[0];
        out->momentum[1] = r[1];
        out->momentum[2] = r[2];
        out->e_kin = r[3];
        out->e_pot = r[4];
        out->e_int = r[5];
        out->front = r[6];
        out->max_drho = r[7];
        out->t = hctrl->t;
        out->n_substeps = hctrl->nsub_total;
        out->n_steps = hctrl->steps_done;
        return SPHX_OK;
    }

    int profile(int32_t reps, double* ms) override
    {
        if (!configured) return ctx->fail(SPHX_ESTATE, "no neighbour configuration");
        if (reps < 1 || !ms) return ctx->fail(SPHX_EINVAL, "bad profile arguments");
        RETCHK(sync_ctrl());
        Ctrl saved = *hctrl;
        RETCHK(backup_state());
        hipEvent_t ev[2];
        HIPCHK(hipEventCreate(&ev[0]));
        HIPCHK(hipEventCreate(&ev[1]));
        double dt_ac = P.cfl_ac_h / (P.c0d + hctrl->vmax);
        hctrl->ss[0] = SubState{0.0, dt_ac, 0, 1, 0, 0};
        hctrl->err = 0;
        RETCHK(push_ctrl());
        float t;
        // pressure relaxation
        HIPCHK(hipEventRecord(ev[0], s));
        for (int r = 0; r < reps; ++r)
            k_pressure<D, real, LN><<<nblk((long long)nf * LN), BLOCK, 0, s>>>(
                P, ctrl, geo[cur], wgeo, wnrm, nbr, ncnt, wnb, wcnt, st[cur], dr3[cur], hf, nullptr, 0, 0, vslot);
        HIPCHK(hipEventRecord(ev[1], s));
        HIPCHK(hipEventSynchronize(ev[1]));
        HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
        ms[0] = t / reps;
        // density relaxation (with its |v|max reduction and clock update)
        HIPCHK(hipEventRecord(ev[0], s));
        for (int r = 0; r < reps; ++r)
            k_density<D, real, LN><<<nblk((long long)nf * LN), BLOCK, 0, s>>>(P, ctrl, 1, geo[cur], wgeo, wnrm, nbr, ncnt, wnb, wcnt, hf,
                                                           st[cur], dr3[cur], x[cur][0], x[cur][1], x[cur][2], nullptr,
                                                                         vslot, 0);
        HIPCHK(hipEventRecord(ev[1], s));
        HIPCHK(hipEventSynchronize(ev[1]));
        HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
        ms[1] = t / reps;
        // neighbour build (idempotent on the current set)
        HIPCHK(hipEventRecord(ev[0], s));
        for (int r = 0; r < reps; ++r)
            k_neighbors<D, real, LN, LB><<<nblk((long long)nf * LB), BLOCK, 0, s>>>(
                P, ctrl, 0, x[cur][0], x[cur][1], x[cur][2], cell[cur], fstart, geo[cur], wx[0], wx[1], wx[2], wstart,
                wgeo, nbr, ncnt, wnb, wcnt);
        HIPCHK(hipEventRecord(ev[1], s));
        HIPCHK(hipEventSynchronize(ev[1]));
        HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
        ms[2] = t / reps;
        // density re-initialisation (gate off; restored below)
        HIPCHK(hipEventRecord(ev[0], s));
        for (int r = 0; r < reps; ++r)
            k_reinit<D, real, LN><<<nblk((long long)nf * LN), BLOCK, 0, s>>>(P, ctrl, 0, geo[cur], wgeo, nbr, ncnt, wnb, wcnt, st[cur]);
        HIPCHK(hipEventRecord(ev[1], s));
        HIPCHK(hipEventSynchronize(ev[1]));
        HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
        ms[3] = t / reps;
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        HIPCHK(hipGetLastError());
        RETCHK(sync_ctrl());
        uint32_t e = hctrl->err;
        RETCHK(restore_state(saved));
        return err_code(e);
    }

    int counts(int64_t* out) override
    {
        if (!out) return ctx->fail(SPHX_EINVAL, "NULL output");
        out[0] = nf;
        out[1] = nw;
        out[2] = out[3] = 0;
        if (!configured || nf == 0) return SPHX_OK;
        std::vector<int32_t> a(nf), b(nf);
        HIPCHK(hipMemcpyAsync(a.data(), ncnt, sizeof(int32_t) * nf, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(b.data(), wcnt, sizeof(int32_t) * nf, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int i = 0; i < nf; ++i) {
            out[2] += a[i];
            out[3] += b[i];
        }
        return SPHX_OK;
    }
};

// ---------------------------------------------------------------------
// C ABI

extern "C" {

int sphx_create(const sphx_params* params, void* stream, sphx_ctx** out)
{
    if (!params || !out) return SPHX_EINVAL;
    *out = nullptr;
    const sphx_params& q = *params;
    if ((q.dim != 2 && q.dim != 3) || (q.precision != SPHX_FP32 && q.precision != SPHX_FP64) || !(q.dp > 0) ||
        !(q.h > 0) || !(q.rho0 > 0) || !(q.c0 > 0) || !(q.u_ref > 0) || !(q.cfl_ad > 0) || !(q.cfl_ac > 0))
        return SPHX_EINVAL;
    std::unique_ptr<sphx_ctx> ctx(new (std::nothrow) sphx_ctx());
    if (!ctx) return SPHX_ENOMEM;
    ctx->prm = q;
    if (stream) {
        ctx->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return SPHX_EHIP;
        ctx->own_stream = true;
    }
    if (q.dim == 2 && q.precision == SPHX_FP64) ctx->eng.reset(new Engine<2, double>(ctx.get()));
    else if (q.dim == 2) ctx->eng.reset(new Engine<2, float>(ctx.get()));
    else if (q.precision == SPHX_FP64) ctx->eng.reset(new Engine<3, double>(ctx.get()));
    else ctx->eng.reset(new Engine<3, float>(ctx.get()));
    int rc = ctx->eng->init();
    if (rc != SPHX_OK) {
        ctx->eng.reset();
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
        return rc;
    }
    *out = ctx.release();
    return SPHX_OK;
}

void sphx_destroy(sphx_ctx* ctx)
{
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    ctx->eng.reset();
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

const char* sphx_last_error(const sphx_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

#define ENG_CALL(expr)                  \
    do {                                \
        if (!ctx) return SPHX_EINVAL;   \
        ctx->err.clear();               \
        return ctx->eng->expr;          \
    } while (0)

int sphx_set_fluid(sphx_ctx* ctx, int64_t n, const double* pos, const double* vel, const double* rho, const double* drho)
{
    ENG_CALL(set_fluid(n, pos, vel, rho, drho));
}

int sphx_set_walls(sphx_ctx* ctx, int64_t n, const double* pos, const double* normal)
{
    ENG_CALL(set_walls(n, pos, normal));
}

int sphx_build_neighbors(sphx_ctx* ctx) { ENG_CALL(build_neighbors()); }

int sphx_get_neighbors(sphx_ctx* ctx, int kind, int64_t* off, int64_t* idx, int64_t cap, int64_t* n_out)
{
    if (ctx && kind != SPHX_INNER && kind != SPHX_CONTACT) return ctx->fail(SPHX_EINVAL, "bad neighbour kind");
    ENG_CALL(get_neighbors(kind, off, idx, cap, n_out));
}

int sphx_density_reinit(sphx_ctx* ctx) { ENG_CALL(density_reinit()); }

int sphx_time_steps(sphx_ctx* ctx, double* dt_ad, double* dt_ac) { ENG_CALL(time_steps(dt_ad, dt_ac)); }

int sphx_compute_rates(sphx_ctx* ctx, double dt, double* dvdt, double* drhodt)
{
    ENG_CALL(compute_rates(dt, dvdt, drhodt));
}

int sphx_advance(sphx_ctx* ctx, int32_t n_steps, double t_stop, int64_t* n_substeps, double* t_out)
{
    ENG_CALL(advance(n_steps, t_stop, n_substeps, t_out));
}

int sphx_get_field(sphx_ctx* ctx, int field, double* out) { ENG_CALL(get_field(field, out)); }

int sphx_diagnostics(sphx_ctx* ctx, sphx_diag* out) { ENG_CALL(diagnostics(out)); }

int sphx_profile(sphx_ctx* ctx, int32_t reps, double* ms) { ENG_CALL(profile(reps, ms)); }

int sphx_counts(sphx_ctx* ctx, int64_t* out) { ENG_CALL(counts(out)); }

}  // extern "C"
