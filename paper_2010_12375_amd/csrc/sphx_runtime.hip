// sphx_runtime.hip -- host runtime of the MI355X Riemann-WCSPH library:
// context, batch layout of the cases, device buffers, HIP-graph capture of
// the advection step and the C ABI declared in include/sphx.h. All particle
// arithmetic runs in the kernels of sphx_device.hpp; the host only sizes
// buffers, launches, captures graphs and marshals arrays in and out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "sphx.h"
#include "sphx_device.hpp"
#include "sphx_gnn.hpp"

using namespace sphx;

struct EngineBase;

// Scratch of the allocation-free diagnostics (sphx_diagnostics_noalloc): a
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes `scratch` itself to a kernel (its host-side name is
// not a device address): each device's address comes from
// hipGetSymbolAddress, taken once per device at context creation with that
// device current, and kept in scratch_addr.
constexpr size_t SCRATCH_DOUBLES = (size_t)1 << 19;  // 4 MiB per GPU
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];
constexpr int SCRATCH_MAX_DEVICES = 64;
static double* scratch_addr[SCRATCH_MAX_DEVICES] = {};
static std::mutex scratch_mu;

// Address of the current device's scratch (taken on first use per device).
static hipError_t scratch_for_device(int dev, double** out)
{
    *out = nullptr;
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_addr[dev] = (double*)p;
    }
    *out = scratch_addr[dev];
    return hipSuccess;
}

struct sphx_ctx {
    std::vector<sphx_params> prm;
    hipStream_t stream = nullptr;
    int device = -1;  // current device at creation (the context's GPU)
    bool own_stream = false;
    std::string err;
    std::unique_ptr<EngineBase> eng;
    int fail(int code, const std::string& msg)
    {
        err = msg;
        return code;
    }
    // (a literal into the capacity reserved at creation: no allocation for
    // messages shorter than that)
    int fail(int code, const char* msg)
    {
        err.assign(msg);
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
    virtual int ncases() const = 0;
    virtual int set_fluid(int c, int64_t n, const double* pos, const double* vel, const double* rho,
                          const double* drho) = 0;
    virtual int set_walls(int c, int64_t n, const double* pos, const double* nrm) = 0;
    virtual int set_wall_motion(int c, const sphx_wall_motion* m, const int32_t* moving) = 0;
    virtual int set_wall_velocity(int c, const double* vel) = 0;
    virtual int save(const char* path) = 0;
    virtual int load(const char* path) = 0;
    virtual int set_fluid_device(int c, int64_t n, const double* pos, const double* vel, const double* rho,
                                 const double* drho) = 0;
    virtual int get_field_device(int c, int which, double* out) = 0;
    virtual int build_neighbors() = 0;
    virtual int get_neighbors(int c, int kind, int64_t* off, int64_t* idx, int64_t cap, int64_t* n_out) = 0;
    virtual int density_reinit() = 0;
    virtual int time_steps(int c, double* dt_ad, double* dt_ac) = 0;
    virtual int compute_rates(int c, double dt, double* dvdt, double* drhodt) = 0;
    virtual int advance(int32_t n_steps, double t_stop, int64_t* nsub, double* t_out) = 0;
    virtual int case_status(int c) = 0;
    virtual int get_field(int c, int which, double* out) = 0;
    virtual int diagnostics(int c, sphx_diag* out) = 0;
    virtual int diagnostics_noalloc(int c, sphx_diag* out) = 0;
    virtual int profile(int32_t reps, double* ms) = 0;
    virtual int counts(int c, int64_t* out) = 0;
    virtual int autotune(int32_t reps, int32_t* lanes, double* times) = 0;
    virtual int set_lanes(int32_t lanes) = 0;
    virtual int set_params_case(int c, const sphx_params* q) = 0;
    virtual int gnn_set_params(const float* p, int64_t n) = 0;
    virtual int gnn_get(int which, float* p, int64_t n) = 0;
    virtual int gnn_forward() = 0;
    virtual int gnn_get_output(int c, double* out) = 0;
    virtual int gnn_set_target(int c, const double* t) = 0;
    virtual int gnn_train_step(double lr, double* loss) = 0;
    virtual int gnn_profile(int32_t reps, double* ms, int64_t* sizes) = 0;
    virtual int surrogate_advance(int32_t windows, double max_drho, int32_t plain_every, int64_t* n_fallback,
                                  int64_t* n_surrogate) = 0;
};

// Parameter layout of the surrogate (float offsets into the flat array, in
// storage order) and of its bf16 weight copies (K x 64 elements each).
struct GnnLayout {
    int Wn, bn, We, be, Wa[3], Wb[3], Wc[3], bm[3], qw[3], Wu[3], bu[3], Wo1, bo1, Wo2, bo2, total;
    int pWn, pWe, pWa[3], pWb[3], pWc[3], pWu[3], pWo1, ptotal;
    GnnLayout()
    {
        int o = 0, q = 0;
        auto take = [&](int n) { int r = o; o += n; return r; };
        auto pk = [&](int k) { int r = q; q += k * gnn::HID; return r; };
        Wn = take(32 * 64); bn = take(64); We = take(32 * 64); be = take(64);
        pWn = pk(32); pWe = pk(32);
        for (int l = 0; l < 3; ++l) {
            Wa[l] = take(64 * 64); Wb[l] = take(64 * 64); Wc[l] = take(64 * 64); bm[l] = take(64); qw[l] = take(64);
            Wu[l] = take(128 * 64); bu[l] = take(64);
            pWa[l] = pk(64); pWb[l] = pk(64); pWc[l] = pk(64); pWu[l] = pk(128);
        }
        Wo1 = take(64 * 64); bo1 = take(64); Wo2 = take(64 * 3); bo2 = take(3);
        pWo1 = pk(64);
        total = o;
        ptotal = q;
    }
};

static inline int nblk(long long n) { return (int)((n + BLOCK - 1) / BLOCK); }
static inline int round_tile(long long n) { return (int)((n + TILE - 1) / TILE * TILE); }

template <int D, typename real>
struct Engine final : EngineBase {
    using G = typename GeoSel<D, real>::T;
    sphx_ctx* ctx;
    hipStream_t s;
    // lanes per particle in the neighbour build (one tile per block): the 3D
    // rows, trimmed to the x sub-bins in reach, are short enough for two
    static constexpr int LB = D == 3 ? 2 : 4;
    int ln = D == 2 ? 4 : 8;      // lanes per particle in the pair kernels (2, 4, 8 or 16)
    int C = 0;                    // cases
    std::vector<KP<real>> hP;     // parameter table (host copy)
    KP<real>* dP = nullptr;
    int32_t* tcase = nullptr;     // case of every tile
    int ntiles = 0, ntot = 0;     // tiles and fluid slots of the layout
    int ncell = 0;                // cells of all cases, padding cells included
    int nsub_q = 5, steps_per_graph = 2;
    int maxn = 0, maxw = 0;
    bool laid_out = false;
    // fluid: two state sets (current and placement target)
    double* x[2][3] = {};
    R4<real>* st[2] = {};
    real* dr3[2] = {};
    G* geo[2] = {};
    int32_t* id[2] = {};
    int32_t* cell[2] = {};
    R4<real>* hf = nullptr;
    R4<real>* avt = nullptr;  // per particle: shear and transport accelerations of the advection step
    uint32_t* nbr = nullptr;
    int32_t* ncnt = nullptr;
    uint32_t* wnb = nullptr;
    int32_t* wcnt = nullptr;
    int32_t *key = nullptr, *rank = nullptr, *perm = nullptr;
    int32_t *cnt = nullptr, *fstart = nullptr, *bsum = nullptr;
    uint32_t* xcum = nullptr;  // per cell: cumulative x sub-bin counts of its fluid particles
    // single-pass scan: per-tile status words, ticket counter, epoch, fault flag
    unsigned long long* lb_status = nullptr;
    int32_t *lb_ticket = nullptr, *lb_fault = nullptr;
    uint32_t* lb_epoch = nullptr;
    real* acc_out = nullptr;
    real* drho_out = nullptr;
    double* outbuf = nullptr;
    double* stage = nullptr;
    size_t stage_n = 0;
    double* diag_part = nullptr;
    double* diag_out = nullptr;
    unsigned long long* vslot = nullptr;  // |v| maxima slots per case (zero between uses)
    // state backup for calls that must leave the state unchanged
    R4<real>* bk_st = nullptr;
    real* bk_dr = nullptr;
    G* bk_geo = nullptr;  // 3D: the frozen geometry carries the density rate in w
    double* bk_x[3] = {};
    // fluid given before the first device layout, per case (uploaded together)
    struct Pending {
        bool has = false;
        std::vector<double> pos, vel, rho, drho;
    };
    std::vector<Pending> pend;
    // walls, all cases concatenated: as given (reference pose, input order)
    // and cell-sorted in the pose of the last configuration update
    int nw_tot = 0;
    std::vector<std::vector<double>> wpos_h, wnrm_h;  // per case, as given
    std::vector<std::vector<int32_t>> wflag_h;         // per case: follows the motion (empty: all)
    std::vector<std::vector<double>> wvel_h;           // per case: given velocities, n*D (empty: none)
    double* wref[6] = {};                              // reference positions and normals, input order
    int32_t *wflag = nullptr, *wcase = nullptr, *wkey = nullptr, *wrank = nullptr, *wperm = nullptr;
    double* wx[3] = {};
    G* wgeo = nullptr;
    G* wnrm = nullptr;
    R4<real>* wmot = nullptr;  // motion records (only while some case has moving walls)
    double* wvin = nullptr;    // given velocities, 3 per wall particle, input order (only while some case has them)
    R4<real>* wvg = nullptr;   // the same in the sorted order
    int32_t* wid = nullptr;
    int32_t* wstart = nullptr;
    // control
    Ctrl* ctrl = nullptr;
    Ctrl* hctrl = nullptr;  // pinned mirror
    int cur = 0;
    bool configured = false;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};  // steps_per_graph queues, by start parity
    hipGraphExec_t gone[2] = {nullptr, nullptr};   // one queue, by start parity
    std::vector<void*> fluid_allocs, wall_allocs;

    Engine(sphx_ctx* c, int ncase) : ctx(c), s(c->stream), C(ncase) {}

    ~Engine() override
    {
        drop_graphs();
        free_list(fluid_allocs);
        free_list(wall_allocs);
        free_list(gn.fixed);
        free_list(gn.nodes);
        free_list(gn.edges);
        for (void* p : {(void*)lb_status, (void*)lb_ticket, (void*)lb_fault, (void*)lb_epoch})
            if (p) (void)hipFree(p);
        for (void* p : {(void*)ctrl, (void*)cnt, (void*)fstart, (void*)xcum, (void*)bsum, (void*)wstart, (void*)diag_out,
                        (void*)dP, (void*)vslot, (void*)stage})
            (void)hipFree(p);
        if (hctrl) (void)hipHostFree(hctrl);
    }

    int ncases() const override { return C; }

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

    std::string case_tag(int c) const { return C > 1 ? "case " + std::to_string(c) + ": " : std::string(); }

    // ------------------------------------------------------------------
    int init_case(int c, int cbase)
    {
        const sphx_params& q = ctx->prm[c];
        KP<real>& P = hP[c];
        P = KP<real>{};
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
        P.s_r = (real)(-0.5 / h);
        P.dWr = (real)(-5.0 * alpha / std::pow(h, D + 2));
        P.quarter_c = (real)(0.25 * q.c0);
        for (int k = 0; k < 3; ++k) P.g[k] = (real)(k < D ? q.gravity[k] : 0.0);
        double rc = 2.0 * h;
        long long nc = 1;
        for (int k = 0; k < 3; ++k) {
            if (k < D) {
                double len = q.hi[k] - q.lo[k];
                if (!(len > 0)) return ctx->fail(SPHX_EINVAL, case_tag(c) + "empty domain box");
                long long n = (long long)std::floor(len / rc);
                while (n > 1 && len / (double)n < rc) --n;
                if (n < 1) n = 1;
                if (n > 100000) return ctx->fail(SPHX_EINVAL, case_tag(c) + "cell grid too large");
                if (q.periodic[k] && n < 3)
                    return ctx->fail(SPHX_EINVAL, case_tag(c) + "a periodic axis needs at least 3 cells of size 2h");
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
            nc *= P.n[k];
        }
        if (nc > 50000000LL || (long long)cbase + nc + 1 > 200000000LL)
            return ctx->fail(SPHX_EINVAL, case_tag(c) + "cell grid too large");
        // cell order: bands of 8 rows along y in 3D (a band's z-neighbour
        // rows then lie 8 x-rows apart), plain row-major in 2D
        P.band = (D == 3 && P.n[1] > 8) ? 8 : P.n[1];
        P.rc2 = (2.0 * h) * (2.0 * h);
        if (q.sigma0 > 0) {
            P.sigma0 = q.sigma0;
        } else {
            // lattice sum of W over the dp lattice, self included
            int K = (int)std::ceil(2.0 * h / q.dp) + 1;
            double sum = 0.0;
            for (int a = -K; a <= K; ++a)
                for (int b = -K; b <= K; ++b)
                    for (int cc = (D == 3 ? -K : 0); cc <= (D == 3 ? K : 0); ++cc) {
                        double r = q.dp * std::sqrt((double)(a * a + b * b + cc * cc));
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
        P.maxn = maxn;
        P.maxw = maxw;
        // the build skips fluid candidates by x sub-bin where the cell width
        // exceeds 2h by more than the rounding of the cell coordinate
        P.xsub_margin = P.Ld[0] > rc * (1.0 + 1e-9) ? 0 : 1;
        if (!(q.eta >= 0.0) || !std::isfinite(q.eta) || !std::isfinite(q.p_background))
            return ctx->fail(SPHX_EINVAL, case_tag(c) + "bad viscosity or background pressure");
        P.eta = (real)q.eta;
        P.p0 = (real)q.p_background;
        P.visc_dt = q.eta > 0.0 ? q.cfl_ad * h * h / (q.eta / q.rho0) : 0.0;
        P.reinit_mode = q.reinit_mode ? 1 : 0;
        P.adv_forces = (q.eta > 0.0 || q.p_background != 0.0) ? 1 : 0;
        P.case_id = c;
        P.cbase = cbase;
        P.ncell = (int)nc;
        return SPHX_OK;
    }

    int init() override
    {
        maxn = D == 2 ? 48 : 128;
        maxw = D == 2 ? 32 : 96;
        hP.resize(C);
        pend.assign(C, Pending{});
        wpos_h.assign(C, {});
        wnrm_h.assign(C, {});
        wflag_h.assign(C, {});
        wvel_h.assign(C, {});
        int cbase = 0;
        for (int c = 0; c < C; ++c) {
            RETCHK(init_case(c, cbase));
            cbase += hP[c].ncell + 1;  // + padding cell
        }
        ncell = cbase;
        nsub_q = ctx->prm[0].nsub_queue > 0 ? ctx->prm[0].nsub_queue : 5;
        if (nsub_q > 64) nsub_q = 64;
        HIPCHK(hipMalloc((void**)&ctrl, sizeof(Ctrl) * C));
        HIPCHK(hipHostMalloc((void**)&hctrl, sizeof(Ctrl) * C, hipHostMallocDefault));
        std::memset(hctrl, 0, sizeof(Ctrl) * C);
        HIPCHK(hipMemcpyAsync(ctrl, hctrl, sizeof(Ctrl) * C, hipMemcpyHostToDevice, s));
        HIPCHK(hipMalloc((void**)&dP, sizeof(KP<real>) * C));
        HIPCHK(hipMalloc((void**)&vslot, sizeof(unsigned long long) * 2 * VSLOTS * C));
        HIPCHK(hipMemsetAsync(vslot, 0, sizeof(unsigned long long) * 2 * VSLOTS * C, s));
        HIPCHK(hipMalloc((void**)&cnt, sizeof(int32_t) * (size_t)ncell));
        HIPCHK(hipMalloc((void**)&fstart, sizeof(int32_t) * ((size_t)ncell + 1)));
        HIPCHK(hipMalloc((void**)&xcum, sizeof(uint32_t) * (size_t)ncell));
        HIPCHK(hipMalloc((void**)&wstart, sizeof(int32_t) * ((size_t)ncell + 1)));
        HIPCHK(hipMalloc((void**)&bsum, sizeof(int32_t) * ((size_t)nblk_scan() + 1)));
        HIPCHK(hipMalloc((void**)&lb_status, sizeof(unsigned long long) * (size_t)nblk_lb()));
        HIPCHK(hipMalloc((void**)&lb_ticket, sizeof(int32_t)));
        HIPCHK(hipMalloc((void**)&lb_fault, sizeof(int32_t)));
        HIPCHK(hipMalloc((void**)&lb_epoch, sizeof(uint32_t)));
        HIPCHK(hipMemsetAsync(lb_status, 0, sizeof(unsigned long long) * (size_t)nblk_lb(), s));
        HIPCHK(hipMemsetAsync(lb_ticket, 0, sizeof(int32_t), s));
        HIPCHK(hipMemsetAsync(lb_fault, 0, sizeof(int32_t), s));
        {
            const uint32_t one = 1u;  // status words of epoch 0 (zeroed) read as empty
            HIPCHK(hipMemcpyAsync(lb_epoch, &one, sizeof(uint32_t), hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        HIPCHK(hipMalloc((void**)&diag_out, sizeof(double) * NDIAG * C));
        HIPCHK(hipMemsetAsync(wstart, 0, sizeof(int32_t) * ((size_t)ncell + 1), s));
        HIPCHK(hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)ncell, s));
        HIPCHK(hipMemsetAsync(xcum, 0, sizeof(uint32_t) * (size_t)ncell, s));
        RETCHK(upload_params());
        HIPCHK(hipStreamSynchronize(s));
        return SPHX_OK;
    }

    int nblk_scan() const { return (ncell + SCAN_TILE - 1) / SCAN_TILE; }
    int nblk_lb() const { return (ncell + LB_TILE - 1) / LB_TILE; }
    int pair_blocks() const { return (int)((long long)ntot * ln / (ln * TILE < BLOCK ? ln * TILE : BLOCK)); }
    template <int T>
    int pair_blocks_t() const { return (int)((long long)ntot * T / pair_threads<T>()); }
    // Lanes of the pressure relaxation for lists laid out for T lanes: in 3D
    // with 8 layout lanes it runs with 4 (its gathers and shuffles favour
    // fewer lanes than the density relaxation's).
    template <int T>
    static constexpr int pressure_lanes() { return D == 3 && T == 8 ? 4 : T; }

    // Whether any case has a shear force or a transport-velocity correction.
    bool any_adv() const
    {
        for (int c = 0; c < C; ++c)
            if (hP[c].adv_forces) return true;
        return false;
    }
    R4<real>* avt_arg() const { return any_adv() ? avt : nullptr; }

    // Whether any case has moving walls.
    bool any_move() const
    {
        for (int c = 0; c < C; ++c)
            if (hP[c].wmove) return true;
        return false;
    }
    R4<real>* wmot_arg() const { return any_move() ? wmot : nullptr; }

    // Whether any case has walls with given velocities.
    bool any_wvel() const
    {
        for (int c = 0; c < C; ++c)
            if (hP[c].wvel) return true;
        return false;
    }
    R4<real>* wvg_arg() const { return any_wvel() ? wvg : nullptr; }

    // Call f with whether the pair kernels need the wall-velocity terms (a
    // motion or given velocities) as a constant (the static instantiation
    // carries none of their code).
    template <typename F>
    void by_motion(F&& f)
    {
        if (any_move() || any_wvel()) f(std::true_type{});
        else f(std::false_type{});
    }

    // Call f with the lanes per particle of the pair kernels as a constant
    // (2, 4 or 8 in 2D; 4, 8 or 16 in 3D: only these are instantiated).
    template <typename F>
    void by_lanes(F&& f)
    {
        if constexpr (D == 2) {
            if (ln == 2) f(std::integral_constant<int, 2>{});
            else if (ln == 4) f(std::integral_constant<int, 4>{});
            else f(std::integral_constant<int, 8>{});
        } else {
            if (ln == 4) f(std::integral_constant<int, 4>{});
            else if (ln == 8) f(std::integral_constant<int, 8>{});
            else f(std::integral_constant<int, 16>{});
        }
    }

    int upload_params()
    {
        HIPCHK(hipMemcpyAsync(dP, hP.data(), sizeof(KP<real>) * C, hipMemcpyHostToDevice, s));
        return SPHX_OK;
    }

    int sync_ctrl()
    {
        int32_t fault = 0;
        HIPCHK(hipMemcpyAsync(hctrl, ctrl, sizeof(Ctrl) * C, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(&fault, lb_fault, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (fault) return ctx->fail(SPHX_EHIP, "cell-count scan: look-back wait exceeded its bound");
        bool fold = false;
        for (int c = 0; c < C; ++c)
            if (hctrl[c].err_pending) {  // raised outside a sub-step queue (rates, profiling)
                hctrl[c].err |= hctrl[c].err_pending;
                hctrl[c].err_pending = 0;
                fold = true;
            }
        if (fold) {
            RETCHK(push_ctrl());
            HIPCHK(hipStreamSynchronize(s));
        }
        return SPHX_OK;
    }

    int push_ctrl()
    {
        HIPCHK(hipMemcpyAsync(ctrl, hctrl, sizeof(Ctrl) * C, hipMemcpyHostToDevice, s));
        return SPHX_OK;
    }

    int err_code(int c, uint32_t e)
    {
        if (e & ERR_NAN) return ctx->fail(SPHX_ENAN, case_tag(c) + "NaN in the particle state");
        if (e & ERR_ESCAPE) return ctx->fail(SPHX_EESCAPE, case_tag(c) + "a fluid particle left the domain box");
        if (e & ERR_NBR_OVERFLOW) return ctx->fail(SPHX_EOVERFLOW, case_tag(c) + "neighbour list capacity exceeded");
        return SPHX_OK;
    }

    // First error among the cases (lowest case index), from the host mirror.
    int first_error()
    {
        for (int c = 0; c < C; ++c)
            if (hctrl[c].err) return err_code(c, hctrl[c].err);
        return SPHX_OK;
    }

    int check_case(int c)
    {
        if (c < 0 || c >= C) return ctx->fail(SPHX_EINVAL, "case index out of range");
        return SPHX_OK;
    }

    int all_have_fluid()
    {
        for (int c = 0; c < C; ++c)
            if (hP[c].nf == 0) return ctx->fail(SPHX_ESTATE, case_tag(c) + "no fluid particles");
        return SPHX_OK;
    }

    // ------------------------------------------------------------------
    // Layout: every case owns hP[c].fcap slots (whole tiles), in case order.
    // With `keep`, the state of every case in the old layout moves to its
    // new slots (case `skip` excepted).
    int layout(bool keep, int skip)
    {
        HIPCHK(hipStreamSynchronize(s));
        std::vector<KP<real>> old = hP;
        double* ox[3] = {x[cur][0], x[cur][1], x[cur][2]};
        R4<real>* ost = st[cur];
        real* odr = dr3[cur];
        int32_t* oid = id[cur];
        int32_t* ocell = cell[cur];
        long long slots = 0;
        for (int c = 0; c < C; ++c) slots += hP[c].fcap;
        if (slots > (long long)CELL_MASK)  // slot indices share a word with a sub-bin (k_scatter)
            return ctx->fail(SPHX_EINVAL, "too many particle slots");
        std::vector<void*> old_allocs;
        old_allocs.swap(fluid_allocs);
        int base = 0;
        for (int c = 0; c < C; ++c) {
            hP[c].fbase = base;
            base += hP[c].fcap;
        }
        ntot = base;
        ntiles = ntot / TILE;
        drop_graphs();
        int rc = alloc_fluid();
        if (rc != SPHX_OK) {
            free_list(old_allocs);
            laid_out = false;
            return rc;
        }
        cur = 0;
        if (keep && laid_out) {
            for (int c = 0; c < C; ++c) {
                if (c == skip || old[c].nf == 0) continue;
                size_t n = (size_t)old[c].nf, o = (size_t)old[c].fbase, d = (size_t)hP[c].fbase;
                for (int k = 0; k < D; ++k)
                    HIPCHK(hipMemcpyAsync(x[0][k] + d, ox[k] + o, n * sizeof(double), hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(st[0] + d, ost + o, n * sizeof(R4<real>), hipMemcpyDeviceToDevice, s));
                if (D == 3) HIPCHK(hipMemcpyAsync(dr3[0] + d, odr + o, n * sizeof(real), hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(id[0] + d, oid + o, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
                HIPCHK(hipMemcpyAsync(cell[0] + d, ocell + o, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
            }
        }
        HIPCHK(hipStreamSynchronize(s));
        free_list(old_allocs);
        std::vector<int32_t> tc(std::max(ntiles, 1), 0);
        for (int c = 0; c < C; ++c)
            for (int t = hP[c].fbase / TILE; t < (hP[c].fbase + hP[c].fcap) / TILE; ++t) tc[t] = c;
        HIPCHK(hipMemcpy(tcase, tc.data(), sizeof(int32_t) * tc.size(), hipMemcpyHostToDevice));
        RETCHK(upload_params());
        laid_out = true;
        configured = false;
        ++conf_gen;
        return SPHX_OK;
    }

    // The first device layout: every case at the size of the fluid given so
    // far, all of it uploaded at once.
    int ensure_layout()
    {
        if (laid_out) return SPHX_OK;
        for (int c = 0; c < C; ++c) hP[c].fcap = round_tile(hP[c].nf);
        RETCHK(layout(false, -1));
        for (int c = 0; c < C; ++c) {
            Pending& p = pend[c];
            if (p.has && hP[c].nf > 0)
                RETCHK(load_case(c, hP[c].nf, p.pos.data(), p.vel.empty() ? nullptr : p.vel.data(),
                                 p.rho.empty() ? nullptr : p.rho.data(), p.drho.empty() ? nullptr : p.drho.data()));
            p = Pending{};
        }
        return SPHX_OK;
    }

    int alloc_fluid()
    {
        const int n = std::max(ntot, TILE);
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
        RETCHK(dalloc(L, tcase, n / TILE));
        RETCHK(dalloc(L, hf, n));
        RETCHK(dalloc(L, avt, 2 * (size_t)n));
        RETCHK(dalloc(L, nbr, (size_t)maxn * n));
        RETCHK(dalloc(L, ncnt, n));
        RETCHK(dalloc(L, wnb, (size_t)maxw * n));
        RETCHK(dalloc(L, wcnt, n));
        RETCHK(dalloc(L, key, n));
        RETCHK(dalloc(L, rank, n));
        RETCHK(dalloc(L, perm, n));
        RETCHK(dalloc(L, acc_out, (size_t)n * D));
        RETCHK(dalloc(L, drho_out, n));
        RETCHK(dalloc(L, outbuf, (size_t)n * std::max(D, 3)));  // fields (n x dim) and surrogate outputs (n x 3)
        RETCHK(dalloc(L, diag_part, (size_t)(n / TILE) * NDIAG));
        RETCHK(dalloc(L, bk_st, n));
        if (D == 3) RETCHK(dalloc(L, bk_dr, n));
        if (D == 3) RETCHK(dalloc(L, bk_geo, n));
        for (int k = 0; k < D; ++k) RETCHK(dalloc(L, bk_x[k], n));
        if (D == 2) bk_x[2] = bk_x[1];
        return SPHX_OK;
    }

    int ensure_stage(size_t ndoubles)
    {
        if (ndoubles <= stage_n) return SPHX_OK;
        if (stage) {
            HIPCHK(hipStreamSynchronize(s));
            (void)hipFree(stage);
            stage = nullptr;
            stage_n = 0;
        }
        HIPCHK(hipMalloc((void**)&stage, ndoubles * sizeof(double)));
        stage_n = ndoubles;
        return SPHX_OK;
    }

    // Fluid from device memory (the context's device): staged on the host
    // before the first device layout, copied device to device afterwards.
    int set_fluid_device(int c, int64_t n, const double* pos, const double* vel, const double* rho,
                         const double* drho) override
    {
        RETCHK(check_case(c));
        if (n < 0 || (n > 0 && !pos)) return ctx->fail(SPHX_EINVAL, "bad fluid particle count or positions");
        if (!laid_out || round_tile(n) > hP[c].fcap) {
            const size_t nn = (size_t)n;
            std::vector<double> hp(nn * D), hv(vel ? nn * D : 0), hr(rho ? nn : 0), hd(drho ? nn : 0);
            HIPCHK(hipStreamSynchronize(s));
            if (n > 0) {
                HIPCHK(hipMemcpy(hp.data(), pos, nn * D * sizeof(double), hipMemcpyDeviceToHost));
                if (vel) HIPCHK(hipMemcpy(hv.data(), vel, nn * D * sizeof(double), hipMemcpyDeviceToHost));
                if (rho) HIPCHK(hipMemcpy(hr.data(), rho, nn * sizeof(double), hipMemcpyDeviceToHost));
                if (drho) HIPCHK(hipMemcpy(hd.data(), drho, nn * sizeof(double), hipMemcpyDeviceToHost));
            }
            return set_fluid(c, n, hp.data(), vel ? hv.data() : nullptr, rho ? hr.data() : nullptr,
                             drho ? hd.data() : nullptr);
        }
        return set_fluid_impl(c, n, pos, vel, rho, drho, true);
    }

    int set_fluid(int c, int64_t n, const double* pos, const double* vel, const double* rho,
                  const double* drho) override
    {
        return set_fluid_impl(c, n, pos, vel, rho, drho, false);
    }

    int set_fluid_impl(int c, int64_t n, const double* pos, const double* vel, const double* rho,
                       const double* drho, bool device)
    {
        RETCHK(check_case(c));
        if (n < 0 || (n > 0 && !pos) || n > (int64_t)NBR_MASK / 2)
            return ctx->fail(SPHX_EINVAL, "bad fluid particle count or positions");
        long long others = 0;
        for (int d = 0; d < C; ++d)
            if (d != c) others += laid_out ? hP[d].fcap : round_tile(hP[d].nf);
        if (others + round_tile(n) > (long long)NBR_MASK) return ctx->fail(SPHX_EINVAL, "too many particles in the batch");
        if (!laid_out) {
            // kept on the host until the first call that needs the device
            Pending& p = pend[c];
            p.has = true;
            const size_t nn = (size_t)n;
            p.pos.assign(pos, pos + nn * D);
            if (vel) p.vel.assign(vel, vel + nn * D);
            else p.vel.clear();
            if (rho) p.rho.assign(rho, rho + nn);
            else p.rho.clear();
            if (drho) p.drho.assign(drho, drho + nn);
            else p.drho.clear();
            hP[c].nf = (int)n;
            std::memset(&hctrl[c], 0, sizeof(Ctrl));
            configured = false;
            return SPHX_OK;
        }
        HIPCHK(hipStreamSynchronize(s));
        hP[c].nf = (int)n;
        if (round_tile(n) > hP[c].fcap) {
            hP[c].fcap = round_tile(n);
            RETCHK(layout(true, c));
        } else {
            RETCHK(upload_params());
            configured = false;
        }
        return load_case(c, n, pos, vel, rho, drho, device);
    }

    // Load case c's fluid (n particles, original order) into its slots of the
    // current set; reset its clock and counters and take its |v|max.
    int load_case(int c, int64_t n, const double* pos, const double* vel, const double* rho, const double* drho,
                  bool device = false)
    {
        size_t nn = (size_t)n;
        RETCHK(ensure_stage(nn * (2 * D + 2)));
        double* dpos = stage;
        double* dvel = stage + nn * D;
        double* drh = stage + nn * 2 * D;
        double* ddr = drh + nn;
        const hipMemcpyKind kind = device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        if (n > 0) {
            HIPCHK(hipMemcpyAsync(dpos, pos, nn * D * sizeof(double), kind, s));
            if (vel) HIPCHK(hipMemcpyAsync(dvel, vel, nn * D * sizeof(double), kind, s));
            if (rho) HIPCHK(hipMemcpyAsync(drh, rho, nn * sizeof(double), kind, s));
            if (drho) HIPCHK(hipMemcpyAsync(ddr, drho, nn * sizeof(double), kind, s));
            k_load_fluid<D, real><<<nblk(n), BLOCK, 0, s>>>(dP, c, dpos, vel ? dvel : nullptr, rho ? drh : nullptr,
                                                             drho ? ddr : nullptr, x[cur][0], x[cur][1], x[cur][2],
                                                             st[cur], dr3[cur], id[cur], cell[cur]);
            HIPCHK(hipGetLastError());
        }
        RETCHK(sync_ctrl());
        std::memset(&hctrl[c], 0, sizeof(Ctrl));
        RETCHK(push_ctrl());
        if (n > 0) {
            k_vmax<D, real><<<nblk(ntot), BLOCK, 0, s>>>(dP, tcase, ntiles, c, nullptr, ctrl, st[cur]);
            k_vmax_fin<real><<<(C + 63) / 64, 64, 0, s>>>(ctrl, C, c, nullptr);
            HIPCHK(hipGetLastError());
        }
        return sync_ctrl();
    }

    int set_walls(int c, int64_t n, const double* pos, const double* nrm) override
    {
        RETCHK(check_case(c));
        if (n < 0 || (n > 0 && (!pos || !nrm)) || n > (int64_t)NBR_MASK / 2)
            return ctx->fail(SPHX_EINVAL, "bad wall particle count or arrays");
        const KP<real>& P = hP[c];
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < D; ++k) {
                double v = pos[i * D + k];
                if (!(v >= P.lo[k] && v < P.hi[k]))
                    return ctx->fail(SPHX_EINVAL, case_tag(c) + "wall particle outside the domain box");
            }
        long long tot = 0;
        for (int d = 0; d < C; ++d) tot += d == c ? n : hP[d].nw;
        if (tot > (long long)NBR_MASK) return ctx->fail(SPHX_EINVAL, "too many wall particles in the batch");
        wpos_h[c].assign(pos, pos + n * D);
        wnrm_h[c].assign(nrm, nrm + n * D);
        hP[c].nw = (int)n;
        hP[c].wmove = 0;  // new walls are static until a motion is given
        hP[c].wvel = 0;   // and carry no velocity until one is given
        wflag_h[c].clear();
        wvel_h[c].clear();
        return upload_walls();
    }

    // Given velocities of case c's wall particles (n*D in the order the
    // walls were given; NULL: none). They do not move the walls.
    int set_wall_velocity(int c, const double* vel) override
    {
        RETCHK(check_case(c));
        KP<real>& P = hP[c];
        if (!vel) {
            P.wvel = 0;
            wvel_h[c].clear();
            return upload_walls();
        }
        const size_t m = (size_t)P.nw * D;
        bool any = false;
        for (size_t k = 0; k < m; ++k) {
            if (!std::isfinite(vel[k])) return ctx->fail(SPHX_EINVAL, case_tag(c) + "bad wall velocity");
            any = any || vel[k] != 0.0;
        }
        // all zero: the walls stay at rest (the static code path)
        P.wvel = any ? 1 : 0;
        wvel_h[c].assign(vel, vel + m);
        if (!any) wvel_h[c].clear();
        return upload_walls();
    }

    // Prescribed rigid motion of case c's walls (NULL: static again) and
    // per-wall flags (NULL: every wall particle follows it). The reach of the
    // motion must stay inside the domain box, and no periodic axis may move.
    int set_wall_motion(int c, const sphx_wall_motion* m, const int32_t* moving) override
    {
        RETCHK(check_case(c));
        KP<real>& P = hP[c];
        if (!m) {
            P.wmove = 0;
            wflag_h[c].clear();
            return upload_walls();
        }
        sphx_wall_motion q = *m;
        if (D == 2) q.amp[2] = q.pivot[2] = 0.0;
        bool finite = std::isfinite(q.omega) && q.omega >= 0.0 && std::isfinite(q.roll);
        for (int k = 0; k < 3; ++k) finite = finite && std::isfinite(q.amp[k]) && std::isfinite(q.pivot[k]);
        if (!finite) return ctx->fail(SPHX_EINVAL, case_tag(c) + "bad wall motion");
        for (int k = 0; k < D; ++k)
            if (P.periodic[k] && (q.amp[k] != 0.0 || (k < 2 && q.roll != 0.0)))
                return ctx->fail(SPHX_EINVAL, case_tag(c) + "walls cannot move along a periodic axis");
        const int nw = P.nw;
        std::vector<int32_t> fl(nw, 1);
        if (moving)
            for (int w = 0; w < nw; ++w) fl[w] = moving[w] != 0;
        const std::vector<double>& xp = wpos_h[c];
        for (int w = 0; w < nw; ++w) {
            if (!fl[w]) continue;
            const double* x = &xp[(size_t)w * D];
            double arm = std::hypot(x[0] - q.pivot[0], x[1] - q.pivot[1]);
            for (int k = 0; k < D; ++k) {
                // displacement bound: |amp_k| plus the chord |roll| * arm of the rotation
                double reach = std::fabs(q.amp[k]) + (k < 2 ? std::fabs(q.roll) * arm : 0.0);
                double margin = 1e-12 * (P.hi[k] - P.lo[k]);
                if (!(x[k] - reach >= P.lo[k] + margin && x[k] + reach < P.hi[k] - margin))
                    return ctx->fail(SPHX_EINVAL, case_tag(c) + "the wall motion leaves the domain box");
            }
        }
        // a motion that moves no wall particle leaves the case static
        P.wmove = std::count(fl.begin(), fl.end(), 1) > 0 ? 1 : 0;
        for (int k = 0; k < 3; ++k) {
            P.wamp[k] = q.amp[k];
            P.wpivot[k] = q.pivot[k];
        }
        P.womega = q.omega;
        P.wroll = q.roll;
        wflag_h[c] = fl;
        return upload_walls();
    }

    // Concatenate the walls of every case (reference pose, input order) and
    // sort them by (global) cell and input order in their current pose.
    int upload_walls()
    {
        HIPCHK(hipStreamSynchronize(s));
        drop_graphs();
        configured = false;
        free_list(wall_allocs);
        wmot = nullptr;
        wvin = nullptr;
        wvg = nullptr;
        int base = 0;
        for (int c = 0; c < C; ++c) {
            hP[c].wbase = base;
            base += hP[c].nw;
        }
        nw_tot = base;
        RETCHK(upload_params());
        const int wcap = std::max(nw_tot, 1);
        auto& L = wall_allocs;
        for (int k = 0; k < D; ++k) RETCHK(dalloc(L, wx[k], wcap));
        if (D == 2) wx[2] = wx[1];
        RETCHK(dalloc(L, wgeo, wcap));
        RETCHK(dalloc(L, wnrm, wcap));
        RETCHK(dalloc(L, wid, wcap));
        if (nw_tot == 0) {
            HIPCHK(hipMemsetAsync(wstart, 0, sizeof(int32_t) * ((size_t)ncell + 1), s));
            HIPCHK(hipStreamSynchronize(s));
            return SPHX_OK;
        }
        for (int k = 0; k < 6; ++k) RETCHK(dalloc(L, wref[k], wcap));
        RETCHK(dalloc(L, wflag, wcap));
        RETCHK(dalloc(L, wcase, wcap));
        RETCHK(dalloc(L, wkey, wcap));
        RETCHK(dalloc(L, wrank, wcap));
        RETCHK(dalloc(L, wperm, wcap));
        if (any_move()) RETCHK(dalloc(L, wmot, wcap));
        if (any_wvel()) {
            RETCHK(dalloc(L, wvin, (size_t)3 * wcap));
            RETCHK(dalloc(L, wvg, wcap));
        }
        size_t nn = (size_t)nw_tot;
        std::vector<double> soa(nn * 6, 0.0);
        std::vector<int32_t> wc(nn), wf(nn);
        for (int c = 0; c < C; ++c)
            for (int i = 0; i < hP[c].nw; ++i) {
                size_t g = (size_t)hP[c].wbase + i;
                wc[g] = c;
                wf[g] = wflag_h[c].empty() ? 1 : wflag_h[c][i];
                for (int k = 0; k < D; ++k) {
                    soa[k * nn + g] = wpos_h[c][(size_t)i * D + k];
                    soa[(3 + k) * nn + g] = wnrm_h[c][(size_t)i * D + k];
                }
            }
        for (int k = 0; k < 6; ++k)
            HIPCHK(hipMemcpyAsync(wref[k], soa.data() + k * nn, nn * sizeof(double), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(wcase, wc.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(wflag, wf.data(), nn * sizeof(int32_t), hipMemcpyHostToDevice, s));
        std::vector<double> wv;
        if (wvin) {
            wv.assign(3 * nn, 0.0);
            for (int c = 0; c < C; ++c)
                if (hP[c].wvel)
                    for (int i = 0; i < hP[c].nw; ++i)
                        for (int k = 0; k < D; ++k)
                            wv[3 * ((size_t)hP[c].wbase + i) + k] = wvel_h[c][(size_t)i * D + k];
            HIPCHK(hipMemcpyAsync(wvin, wv.data(), wv.size() * sizeof(double), hipMemcpyHostToDevice, s));
        }
        RETCHK(enqueue_wall_sort());
        HIPCHK(hipStreamSynchronize(s));
        return SPHX_OK;
    }

    // Pose, bin and sort the walls of every case at its clock (the cell
    // counters are consumed and cleared by the scan, so this can sit in a
    // captured graph).
    int enqueue_wall_sort()
    {
        if (nw_tot == 0) return SPHX_OK;
        const int n = nw_tot;
        const int D3 = D == 3 ? 2 : 1;
        k_bin_walls<D, real><<<nblk(n), BLOCK, 0, s>>>(dP, wcase, ctrl, wflag, n, wref[0], wref[1], wref[D3], wkey,
                                                        wrank, cnt);
        RETCHK(enqueue_scan(wstart));
        k_scatter_walls<<<nblk(n), BLOCK, 0, s>>>(n, wkey, wrank, wstart, wperm);
        k_gather_wall<D, real><<<nblk(n), BLOCK, 0, s>>>(dP, wcase, ctrl, wflag, n, wperm, wkey, wstart, wref[0], wref[1],
                                                          wref[D3], wref[3], wref[4], wref[3 + D3], wx[0], wx[1],
                                                          wx[2], wgeo, wnrm, wid, wmot_arg(), wvin, wvg_arg());
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    // Exclusive scan of the cell counts into out[0..ncell]; with q >= 0 the
    // same launch closes the queue's last sub-step q of every case.
    int enqueue_scan(int32_t* out, int q = -1)
    {
        if (nblk_lb() <= LB_MAX_BLOCKS) {
            k_scan_lb<real><<<nblk_lb(), BLOCK, 0, s>>>(cnt, out, ncell, lb_status, lb_ticket, lb_epoch, lb_fault,
                                                         dP, ctrl, vslot, q, C);
        } else {
            const int nb = nblk_scan();
            k_scan_tiles<<<nb, BLOCK, 0, s>>>(cnt, out, bsum, ncell);
            k_scan_fin<real><<<nb, BLOCK, 0, s>>>(out, bsum, ncell, dP, ctrl, vslot, q, C);
        }
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    // S1-S3 from state set a into set b for every case (a full update where
    // a step ended or `force`, the identity elsewhere). The cell counters are
    // zero on entry (zeroed at allocation and by every scan that consumes
    // them).
    template <int T>
    void launch_neighbors(int force, int b, int reinit = 0)
    {
        // with two lanes per particle in the pair kernels (large 2D batches,
        // issue-bound) the build packs two lanes per particle as well
        constexpr int TB = T < LB ? T : LB;
        k_neighbors<D, real, T, TB><<<ntiles, TILE * TB, 0, s>>>(dP, tcase, ctrl, force, x[b][0], x[b][1], x[b][2],
                                                                cell[b], fstart, geo[b], wx[0], wx[1], wx[2], wstart,
                                                                wgeo, nbr, ncnt, wnb, wcnt, reinit, st[b], xcum);
    }

    // `q` >= 0: at the end of a queue whose last sub-step is q (the scan
    // closes it, the binning decides the full updates from the same state).
    // `binned`: the last density relaxation of the queue has done the binning.
    int enqueue_rebuild(int force, int a, int q = -1, bool binned = false)
    {
        ++conf_gen;
        int b = 1 - a;
        const int nb = nblk(ntot);
        if (!binned)
            k_bin<D, real><<<nb, BLOCK, 0, s>>>(dP, tcase, ntiles, ctrl, force, x[a][0], x[a][1], x[a][2], cell[a],
                                                key, rank, cnt, q);
        RETCHK(enqueue_scan(fstart, q));
        if (any_move()) RETCHK(enqueue_wall_sort());  // walls in their pose at each case's (closed) clock
        k_scatter<real><<<nb, BLOCK, 0, s>>>(dP, tcase, ntiles, ntot, key, rank, fstart, perm);
        k_place_fluid<D, real><<<nb, BLOCK, 0, s>>>(dP, tcase, ntiles, ctrl, force, ntot, perm, key, fstart, x[a][0],
                                                     x[a][1], x[a][2], st[a], dr3[a], id[a], geo[a], x[b][0], x[b][1],
                                                     x[b][2], st[b], dr3[b], id[b], cell[b], geo[b], xcum);
        // at the end of a queue the next step's density re-initialisation rides along
        by_lanes([&](auto t) { launch_neighbors<decltype(t)::value>(force, b, q >= 0 ? 1 : 0); });
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    template <int T>
    void launch_substep(int a, int q, int adv, int finalize, real* acc, real* dro, int bin)
    {
        const int nb = pair_blocks();
        R4<real>* av = avt_arg();
        R4<real>* wm = wmot_arg();
        R4<real>* wg = wvg_arg();
        by_motion([&](auto mc) {
            constexpr bool MV = decltype(mc)::value;
            constexpr int TP = pressure_lanes<T>();
            k_pressure<D, real, TP, MV, T><<<pair_blocks_t<TP>(), pair_threads<TP>(), 0, s>>>(
                dP, tcase, ctrl, geo[a], wgeo, wnrm, nbr, ncnt, wnb, wcnt, st[a], dr3[a], hf, acc, q, adv, vslot, av, wm,
                wg);
            k_density<D, real, T, MV><<<nb, pair_threads<T>(), 0, s>>>(dP, tcase, ctrl, finalize, geo[a], wgeo, wnrm, nbr, ncnt,
                                                           wnb, wcnt, hf, st[a], dr3[a], x[a][0], x[a][1], x[a][2],
                                                           dro, vslot, q, av, wm, wg, bin, cell[a], key, rank, cnt);
        });
    }

    // Pressure and density relaxation of sub-step q on set a; `adv`: close
    // sub-step q - 1 first (inside the pressure relaxation).
    int enqueue_substep(int a, int q, int adv, int finalize, real* acc, real* dro, int bin = 0)
    {
        by_lanes([&](auto t) { launch_substep<decltype(t)::value>(a, q, adv, finalize, acc, dro, bin); });
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    int enqueue_reinit(int gate, int a)
    {
        const int nb = pair_blocks();
        by_lanes([&](auto t) {
            k_reinit<D, real, decltype(t)::value><<<nb, pair_threads<decltype(t)::value>(), 0, s>>>(dP, tcase, ctrl, gate, geo[a], wgeo, nbr, ncnt,
                                                                      wnb, wcnt, st[a]);
        });
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    // Shear and transport accelerations of the advection step (after the
    // re-initialisation); `gate`: for the cases starting a step.
    int enqueue_adv_forces(int gate, int a)
    {
        if (!any_adv()) return SPHX_OK;
        const int nb = pair_blocks();
        by_lanes([&](auto t) {
            by_motion([&](auto mc) {
                k_adv_forces<D, real, decltype(t)::value, decltype(mc)::value><<<nb, pair_threads<decltype(t)::value>(), 0, s>>>(
                    dP, tcase, ctrl, gate, geo[a], wgeo, nbr, ncnt, wnb, wcnt, st[a], avt, wmot_arg(), wvg_arg());
            });
        });
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    // One queue on set a (graph body): re-initialisation for the cases
    // starting a step, the queued sub-steps, the step end (which prepares the
    // next step or marks a continuation), the configuration update.
    // One queue: the density re-initialisation (in 2D it came with the
    // configuration update that ended the previous queue, or with advance's
    // prologue) and the advection-step forces of the cases starting a step,
    // the sub-steps, the configuration update.
    int enqueue_step(int a)
    {
        RETCHK(enqueue_adv_forces(1, a));
        for (int q = 0; q < nsub_q; ++q) RETCHK(enqueue_substep(a, q, q > 0, 1, nullptr, nullptr, q == nsub_q - 1));
        RETCHK(enqueue_rebuild(0, a, nsub_q - 1, true));
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
        RETCHK(all_have_fluid());
        RETCHK(ensure_layout());
        RETCHK(sync_ctrl());
        for (int c = 0; c < C; ++c) hctrl[c].err = 0;
        RETCHK(push_ctrl());
        RETCHK(enqueue_rebuild(1, cur));
        RETCHK(sync_ctrl());
        cur ^= 1;
        int rc = first_error();
        if (rc != SPHX_OK) {
            configured = false;
            for (int c = 0; c < C; ++c) hctrl[c].err = 0;
            RETCHK(push_ctrl());
            HIPCHK(hipStreamSynchronize(s));
            return rc;
        }
        configured = true;
        return SPHX_OK;
    }

    size_t ell_index(int i, int k, int mx) const
    {
        return ln == 2 ? ell_at<2>(i, k, mx)
               : ln == 4 ? ell_at<4>(i, k, mx) : ln == 8 ? ell_at<8>(i, k, mx) : ell_at<16>(i, k, mx);
    }

    int get_neighbors(int c, int kind, int64_t* off, int64_t* idx, int64_t cap_idx, int64_t* n_out) override
    {
        RETCHK(check_case(c));
        if (!configured) return ctx->fail(SPHX_ESTATE, "no neighbour configuration");
        const KP<real>& P = hP[c];
        const int nf = P.nf, nw = P.nw;
        const int mx = kind == SPHX_INNER ? maxn : maxw;
        std::vector<int32_t> cnts(std::max(nf, 1)), ids(std::max(nf, 1)), oid(std::max(nw, 1));
        // the case's tiles hold one contiguous range of list words
        const size_t e0 = ell_index(P.fbase, 0, mx), ne = (size_t)mx * P.fcap;
        std::vector<uint32_t> ell(std::max<size_t>(ne, 1));
        if (nf > 0) {
            HIPCHK(hipMemcpyAsync(cnts.data(), (kind == SPHX_INNER ? ncnt : wcnt) + P.fbase, sizeof(int32_t) * nf,
                                  hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(ids.data(), id[cur] + P.fbase, sizeof(int32_t) * nf, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(ell.data(), (kind == SPHX_INNER ? nbr : wnb) + e0, sizeof(uint32_t) * ne,
                                  hipMemcpyDeviceToHost, s));
        }
        if (kind != SPHX_INNER && nw > 0)
            HIPCHK(hipMemcpyAsync(oid.data(), wid + P.wbase, sizeof(int32_t) * nw, hipMemcpyDeviceToHost, s));
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
                    uint32_t j = ell[ell_index(P.fbase + i, k, mx) - e0] & NBR_MASK;
                    idx[o + k] = kind == SPHX_INNER ? ids[j - P.fbase] : oid[j - P.wbase];
                }
                std::sort(idx + o, idx + o + cnts[i]);
            }
        }
        return SPHX_OK;
    }

    int density_reinit() override
    {
        if (!configured) return ctx->fail(SPHX_ESTATE, "no neighbour configuration");
        RETCHK(enqueue_reinit(0, cur));
        HIPCHK(hipStreamSynchronize(s));
        return SPHX_OK;
    }

    int time_steps(int c, double* dt_ad, double* dt_ac) override
    {
        RETCHK(check_case(c));
        if (hP[c].nf == 0) return ctx->fail(SPHX_ESTATE, case_tag(c) + "no fluid particles");
        RETCHK(ensure_layout());
        k_vmax<D, real><<<nblk(ntot), BLOCK, 0, s>>>(dP, tcase, ntiles, c, nullptr, ctrl, st[cur]);
        k_vmax_fin<real><<<(C + 63) / 64, 64, 0, s>>>(ctrl, C, c, nullptr);
        HIPCHK(hipGetLastError());
        RETCHK(sync_ctrl());
        const KP<real>& P = hP[c];
        double vmax = hctrl[c].vmax;
        if (dt_ad) {
            *dt_ad = P.cfl_ad_h / std::fmax(vmax, P.u_ref);
            if (P.visc_dt > 0.0) *dt_ad = std::fmin(*dt_ad, P.visc_dt);
        }
        if (dt_ac) *dt_ac = P.cfl_ac_h / (P.c0d + vmax);
        return SPHX_OK;
    }

    int backup_state()
    {
        HIPCHK(hipMemcpyAsync(bk_st, st[cur], sizeof(R4<real>) * ntot, hipMemcpyDeviceToDevice, s));
        if (D == 3) HIPCHK(hipMemcpyAsync(bk_dr, dr3[cur], sizeof(real) * ntot, hipMemcpyDeviceToDevice, s));
        if (D == 3) HIPCHK(hipMemcpyAsync(bk_geo, geo[cur], sizeof(G) * ntot, hipMemcpyDeviceToDevice, s));
        for (int k = 0; k < D; ++k)
            HIPCHK(hipMemcpyAsync(bk_x[k], x[cur][k], sizeof(double) * ntot, hipMemcpyDeviceToDevice, s));
        return SPHX_OK;
    }

    int restore_state(const std::vector<Ctrl>& saved)
    {
        HIPCHK(hipMemcpyAsync(st[cur], bk_st, sizeof(R4<real>) * ntot, hipMemcpyDeviceToDevice, s));
        if (D == 3) HIPCHK(hipMemcpyAsync(dr3[cur], bk_dr, sizeof(real) * ntot, hipMemcpyDeviceToDevice, s));
        if (D == 3) HIPCHK(hipMemcpyAsync(geo[cur], bk_geo, sizeof(G) * ntot, hipMemcpyDeviceToDevice, s));
        for (int k = 0; k < D; ++k)
            HIPCHK(hipMemcpyAsync(x[cur][k], bk_x[k], sizeof(double) * ntot, hipMemcpyDeviceToDevice, s));
        std::memcpy(hctrl, saved.data(), sizeof(Ctrl) * C);
        RETCHK(push_ctrl());
        HIPCHK(hipStreamSynchronize(s));
        return SPHX_OK;
    }

    int compute_rates(int c, double dt, double* dvdt, double* drhodt) override
    {
        RETCHK(check_case(c));
        if (!configured) return ctx->fail(SPHX_ESTATE, "no neighbour configuration");
        RETCHK(sync_ctrl());
        std::vector<Ctrl> saved(hctrl, hctrl + C);
        RETCHK(backup_state());
        for (int d = 0; d < C; ++d) {
            hctrl[d].ss[0] = SubState{0.0, d == c ? dt : 0.0, 0, d == c ? 1 : 0, 0, 0};
            hctrl[d].midstep = 0;
        }
        hctrl[c].err = 0;
        RETCHK(push_ctrl());
        RETCHK(enqueue_adv_forces(0, cur));
        RETCHK(enqueue_substep(cur, 0, 0, 0, acc_out, drho_out));
        const KP<real>& P = hP[c];
        if (dvdt && P.nf > 0) {
            k_unsort_vec<real><<<nblk(P.nf), BLOCK, 0, s>>>(P.fbase, P.nf, D, id[cur], acc_out, outbuf);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(dvdt, outbuf, sizeof(double) * (size_t)P.nf * D, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        if (drhodt && P.nf > 0) {
            k_unsort_vec<real><<<nblk(P.nf), BLOCK, 0, s>>>(P.fbase, P.nf, 1, id[cur], drho_out, outbuf);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(drhodt, outbuf, sizeof(double) * (size_t)P.nf, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        RETCHK(sync_ctrl());
        uint32_t e = hctrl[c].err;
        RETCHK(restore_state(saved));
        return err_code(c, e);
    }

    bool busy(int c) const { return !hctrl[c].err && (hctrl[c].midstep || hctrl[c].ss[0].active); }

    // Queues every case still needs at least: one advection step per queue,
    // bounded by its step target and by the longest possible advection step.
    long long queues_needed() const
    {
        long long need = 0;
        for (int c = 0; c < C; ++c) {
            if (!busy(c)) continue;
            const Ctrl& k = hctrl[c];
            long long r = k.steps_target - k.steps_done;
            double dt_max = hP[c].cfl_ad_h / hP[c].u_ref;
            double by_time = std::ceil((k.t_stop - k.t) / dt_max);
            if (by_time < (double)r) r = (long long)std::max(by_time, 1.0);
            need = std::max(need, std::max(r, 1LL));
        }
        return need;
    }

    int advance(int32_t n_steps, double t_stop, int64_t* nsub_out, double* t_out) override
    {
        if (n_steps < 0) return ctx->fail(SPHX_EINVAL, "negative step count");
        return advance_cases(std::vector<long long>(C, n_steps), t_stop, nsub_out, t_out);
    }

    // Advance case c by up to steps[c] advection steps (0: the case idles).
    int advance_cases(const std::vector<long long>& steps, double t_stop, int64_t* nsub_out, double* t_out)
    {
        RETCHK(all_have_fluid());
        if (!configured) RETCHK(build_neighbors());
        RETCHK(capture_graphs());
        RETCHK(sync_ctrl());
        std::vector<long long> sub0(C);
        for (int c = 0; c < C; ++c) {
            sub0[c] = hctrl[c].nsub_total;
            hctrl[c].t_stop = t_stop;
            hctrl[c].steps_target = hctrl[c].steps_done + steps[c];
        }
        RETCHK(push_ctrl());
        k_adv_begin<real><<<(C + 63) / 64, 64, 0, s>>>(dP, ctrl, C);
        HIPCHK(hipGetLastError());
        // the first step's density re-initialisation, by the same kernel (and
        // so the same arithmetic) that re-initialises the later steps at the
        // end of each queue: the lists are rebuilt unchanged from the current
        // configuration, so how a run is split into calls changes no bit
        by_lanes([&](auto t) { launch_neighbors<decltype(t)::value>(1, cur, 1); });
        HIPCHK(hipGetLastError());
        RETCHK(sync_ctrl());
        // queues in batches of at most 64, one host synchronisation per batch
        for (long long need = queues_needed(); need > 0; need = queues_needed()) {
            long long batch = std::min<long long>(need, 64);
            long long q = 0;
            for (; q + steps_per_graph <= batch; q += steps_per_graph) {
                HIPCHK(hipGraphLaunch(gexec[cur], s));
                cur = (cur + steps_per_graph) & 1;
            }
            for (; q < batch; ++q) {
                HIPCHK(hipGraphLaunch(gone[cur], s));
                cur ^= 1;
            }
            RETCHK(sync_ctrl());
        }
        long long nsub = 0;
        for (int c = 0; c < C; ++c) nsub += hctrl[c].nsub_total - sub0[c];
        if (nsub_out) *nsub_out = nsub;
        if (t_out) *t_out = hctrl[0].t;
        return first_error();
    }

    int case_status(int c) override
    {
        RETCHK(check_case(c));
        RETCHK(sync_ctrl());
        return err_code(c, hctrl[c].err);
    }

    int get_field(int c, int which, double* out) override { return get_field_impl(c, which, out, false); }
    int get_field_device(int c, int which, double* out) override { return get_field_impl(c, which, out, true); }

    int get_field_impl(int c, int which, double* out, bool device)
    {
        RETCHK(check_case(c));
        if (which < 0 || which > 4 || !out) return ctx->fail(SPHX_EINVAL, "bad field");
        RETCHK(ensure_layout());
        const KP<real>& P = hP[c];
        if (P.nf == 0) return SPHX_OK;
        k_unsort_field<D, real><<<nblk(P.nf), BLOCK, 0, s>>>(dP, c, which, id[cur], x[cur][0], x[cur][1], x[cur][2],
                                                              st[cur], dr3[cur], outbuf);
        HIPCHK(hipGetLastError());
        size_t cnt_out = (which <= 1 ? (size_t)D : 1) * P.nf;
        HIPCHK(hipMemcpyAsync(out, outbuf, sizeof(double) * cnt_out,
                              device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return SPHX_OK;
    }

    // ------------------------------------------------------------------
    // Checkpoint: parameters, walls and their motion, clocks and control
    // blocks, and every case's particle state in the current (cell-sorted)
    // slot order. A context created with the same parameters continues from
    // a loaded checkpoint exactly as the saved one would (the configuration
    // is rebuilt from the sorted state, which the stable sort leaves as is).
    static constexpr char CKPT_MAGIC[9] = "SPHXCK02";

    int save(const char* path) override
    {
        if (!path) return ctx->fail(SPHX_EINVAL, "no checkpoint path");
        RETCHK(ensure_layout());
        RETCHK(sync_ctrl());
        FILE* f = std::fopen(path, "wb");
        if (!f) return ctx->fail(SPHX_EINVAL, std::string("cannot write ") + path);
        bool ok = true;
        auto put = [&](const void* p, size_t bytes) { ok = ok && (bytes == 0 || std::fwrite(p, 1, bytes, f) == bytes); };
        const int32_t hdr[4] = {D, (int32_t)sizeof(real), C, ntot};
        put(CKPT_MAGIC, 8);
        put(hdr, sizeof(hdr));
        for (int c = 0; c < C; ++c) {
            const KP<real>& P = hP[c];
            put(&ctx->prm[c], sizeof(sphx_params));
            const int32_t lay[4] = {P.nf, P.fcap, P.fbase, P.nw};
            put(lay, sizeof(lay));
            put(&hctrl[c], sizeof(Ctrl));
            put(wpos_h[c].data(), wpos_h[c].size() * sizeof(double));
            put(wnrm_h[c].data(), wnrm_h[c].size() * sizeof(double));
            const int32_t nfl = (int32_t)wflag_h[c].size();
            put(&nfl, sizeof(nfl));
            put(wflag_h[c].data(), wflag_h[c].size() * sizeof(int32_t));
            const double mo[8] = {P.wamp[0], P.wamp[1], P.wamp[2], P.womega, P.wroll, P.wpivot[0], P.wpivot[1],
                                  P.wpivot[2]};
            put(&P.wmove, sizeof(int32_t));
            put(mo, sizeof(mo));
            const int32_t nwv = (int32_t)wvel_h[c].size();
            put(&nwv, sizeof(nwv));
            put(wvel_h[c].data(), wvel_h[c].size() * sizeof(double));
        }
        const size_t n = (size_t)ntot;
        std::vector<double> hx(n);
        for (int k = 0; k < D; ++k) {
            HIPCHK(hipMemcpy(hx.data(), x[cur][k], n * sizeof(double), hipMemcpyDeviceToHost));
            put(hx.data(), n * sizeof(double));
        }
        std::vector<R4<real>> hs(n);
        HIPCHK(hipMemcpy(hs.data(), st[cur], n * sizeof(R4<real>), hipMemcpyDeviceToHost));
        put(hs.data(), n * sizeof(R4<real>));
        if (D == 3) {
            std::vector<real> hd(n);
            HIPCHK(hipMemcpy(hd.data(), dr3[cur], n * sizeof(real), hipMemcpyDeviceToHost));
            put(hd.data(), n * sizeof(real));
        }
        std::vector<int32_t> hi(n);
        HIPCHK(hipMemcpy(hi.data(), id[cur], n * sizeof(int32_t), hipMemcpyDeviceToHost));
        put(hi.data(), n * sizeof(int32_t));
        ok = (std::fclose(f) == 0) && ok;
        if (!ok) return ctx->fail(SPHX_EINVAL, std::string("write failed: ") + path);
        return SPHX_OK;
    }

    // Sanity of a checkpoint's contents (SPHX_EINVAL with the reason): the
    // particle ids of each case's used slots are a permutation of [0, nf)
    // (they become write indices when fields are returned in original
    // order); positions, particle state, walls and motion are finite; the
    // control block holds a finite, non-negative clock and step state,
    // flags that are 0 or 1, non-negative counters and known error bits.
    template <typename Rec>
    int check_loaded(const std::vector<Rec>& rec, const std::vector<std::vector<double>>& hx,
                     const std::vector<R4<real>>& hs, const std::vector<real>& hd, const std::vector<int32_t>& hi)
    {
        auto bad = [&](int c, const char* what) { return ctx->fail(SPHX_EINVAL, case_tag(c) + "corrupt checkpoint: " + what); };
        auto fin = [](double v) { return std::isfinite(v); };
        const uint32_t known = ERR_ESCAPE | ERR_NAN | ERR_NBR_OVERFLOW;
        for (int c = 0; c < C; ++c) {
            const Rec& r = rec[c];
            const int nf = r.lay[0], base = r.lay[2];
            std::vector<char> seen((size_t)nf, 0);
            for (int i = base; i < base + nf; ++i) {
                const int32_t v = hi[(size_t)i];
                if (v < 0 || v >= nf || seen[(size_t)v]) return bad(c, "particle ids are not a permutation");
                seen[(size_t)v] = 1;
                for (int k = 0; k < D; ++k)
                    if (!fin(hx[k][(size_t)i])) return bad(c, "non-finite position");
                const R4<real>& q = hs[(size_t)i];
                if (!fin((double)q.x) || !fin((double)q.y) || !fin((double)q.z) || !fin((double)q.w))
                    return bad(c, "non-finite particle state");
                if (D == 3 && !fin((double)hd[(size_t)i])) return bad(c, "non-finite density rate");
            }
            for (double v : r.wp)
                if (!fin(v)) return bad(c, "non-finite wall position");
            for (double v : r.wn)
                if (!fin(v)) return bad(c, "non-finite wall normal");
            for (double v : r.wv)
                if (!fin(v)) return bad(c, "non-finite wall velocity");
            for (int32_t v : r.fl)
                if (v != 0 && v != 1) return bad(c, "wall motion flags other than 0 or 1");
            for (double v : r.mo)
                if (!fin(v)) return bad(c, "non-finite wall motion");
            if (r.wmove != 0 && r.wmove != 1) return bad(c, "wall motion switch other than 0 or 1");
            const Ctrl& k = r.k;
            if (!fin(k.t) || k.t < 0.0 || !fin(k.t_end) || k.t_end < 0.0 || std::isnan(k.t_stop) ||
                !fin(k.dt_ad) || k.dt_ad < 0.0 || !fin(k.vmax) || k.vmax < 0.0)
                return bad(c, "clock or time step state");
            for (const SubState& q : k.ss)
                if (!fin(q.tau) || q.tau < 0.0 || !fin(q.dt) || q.dt < 0.0 || (q.last != 0 && q.last != 1) ||
                    (q.active != 0 && q.active != 1) || q.nsub < 0)
                    return bad(c, "sub-step state");
            if ((k.midstep != 0 && k.midstep != 1) || (k.rebuild != 0 && k.rebuild != 1) || k.nsub_total < 0 ||
                k.steps_done < 0 || k.steps_target < 0)
                return bad(c, "step counters");
            if ((k.err & ~known) || (k.err_pending & ~known)) return bad(c, "unknown error bits");
        }
        return SPHX_OK;
    }

    int load(const char* path) override
    {
        if (!path) return ctx->fail(SPHX_EINVAL, "no checkpoint path");
        FILE* f = std::fopen(path, "rb");
        if (!f) return ctx->fail(SPHX_EINVAL, std::string("cannot read ") + path);
        std::unique_ptr<FILE, int (*)(FILE*)> guard(f, &std::fclose);
        bool ok = true;
        auto get = [&](void* p, size_t bytes) { ok = ok && (bytes == 0 || std::fread(p, 1, bytes, f) == bytes); };
        char magic[8];
        int32_t hdr[4];
        get(magic, 8);
        get(hdr, sizeof(hdr));
        if (!ok || std::memcmp(magic, CKPT_MAGIC, 8) != 0) return ctx->fail(SPHX_EINVAL, "not a checkpoint");
        if (hdr[0] != D || hdr[1] != (int32_t)sizeof(real) || hdr[2] != C || hdr[3] < 0 || hdr[3] % TILE)
            return ctx->fail(SPHX_EINVAL, "checkpoint of another dimension, precision or case count");
        struct CaseRec {
            sphx_params q;
            int32_t lay[4];
            Ctrl k;
            std::vector<double> wp, wn;
            std::vector<int32_t> fl;
            int32_t wmove;
            double mo[8];
            std::vector<double> wv;
        };
        std::vector<CaseRec> rec(C);
        int32_t ntot_f = 0;
        for (int c = 0; c < C && ok; ++c) {
            CaseRec& r = rec[c];
            get(&r.q, sizeof(sphx_params));
            get(r.lay, sizeof(r.lay));
            get(&r.k, sizeof(Ctrl));
            if (!ok) break;
            sphx_params a = r.q, b = ctx->prm[c];
            a.nsub_queue = b.nsub_queue = 0;
            if (std::memcmp(&a, &b, sizeof(sphx_params)) != 0)
                return ctx->fail(SPHX_EINVAL, case_tag(c) + "checkpoint parameters differ from the context's");
            if (r.lay[0] < 0 || r.lay[1] != round_tile(r.lay[0]) || r.lay[2] != ntot_f || r.lay[3] < 0 ||
                r.lay[3] > (int32_t)NBR_MASK)
                return ctx->fail(SPHX_EINVAL, "corrupt checkpoint layout");
            ntot_f += r.lay[1];
            r.wp.resize((size_t)r.lay[3] * D);
            r.wn.resize((size_t)r.lay[3] * D);
            get(r.wp.data(), r.wp.size() * sizeof(double));
            get(r.wn.data(), r.wn.size() * sizeof(double));
            int32_t nfl = 0;
            get(&nfl, sizeof(nfl));
            if (!ok || (nfl != 0 && nfl != r.lay[3])) return ctx->fail(SPHX_EINVAL, "corrupt checkpoint walls");
            r.fl.resize(nfl);
            get(r.fl.data(), r.fl.size() * sizeof(int32_t));
            get(&r.wmove, sizeof(int32_t));
            get(r.mo, sizeof(r.mo));
            int32_t nwv = 0;
            get(&nwv, sizeof(nwv));
            if (!ok || (nwv != 0 && nwv != r.lay[3] * D)) return ctx->fail(SPHX_EINVAL, "corrupt checkpoint walls");
            r.wv.resize(nwv);
            get(r.wv.data(), r.wv.size() * sizeof(double));
        }
        if (!ok || ntot_f != hdr[3]) return ctx->fail(SPHX_EINVAL, "truncated or corrupt checkpoint");
        const size_t n = (size_t)hdr[3];
        std::vector<std::vector<double>> hx(D, std::vector<double>(n));
        for (int k = 0; k < D; ++k) get(hx[k].data(), n * sizeof(double));
        std::vector<R4<real>> hs(n);
        get(hs.data(), n * sizeof(R4<real>));
        std::vector<real> hd(D == 3 ? n : 0);
        if (D == 3) get(hd.data(), n * sizeof(real));
        std::vector<int32_t> hi(n);
        get(hi.data(), n * sizeof(int32_t));
        if (!ok) return ctx->fail(SPHX_EINVAL, "truncated checkpoint");
        // Everything below indexes device and host memory by these values:
        // check them all on the host before anything reaches the device.
        RETCHK(check_loaded(rec, hx, hs, hd, hi));
        // layout exactly as saved, state into set 0
        HIPCHK(hipStreamSynchronize(s));
        for (int c = 0; c < C; ++c) {
            hP[c].nf = rec[c].lay[0];
            hP[c].fcap = rec[c].lay[1];
            pend[c] = Pending{};
        }
        laid_out = false;
        RETCHK(layout(false, -1));
        for (int k = 0; k < D; ++k)
            HIPCHK(hipMemcpy(x[0][k], hx[k].data(), n * sizeof(double), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(st[0], hs.data(), n * sizeof(R4<real>), hipMemcpyHostToDevice));
        if (D == 3) HIPCHK(hipMemcpy(dr3[0], hd.data(), n * sizeof(real), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(id[0], hi.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
        for (int c = 0; c < C; ++c) hctrl[c] = rec[c].k;
        RETCHK(push_ctrl());
        HIPCHK(hipStreamSynchronize(s));
        // walls and motions, posed at the restored clocks
        for (int c = 0; c < C; ++c) {
            CaseRec& r = rec[c];
            wpos_h[c] = r.wp;
            wnrm_h[c] = r.wn;
            hP[c].nw = r.lay[3];
            hP[c].wmove = r.wmove ? 1 : 0;
            hP[c].wamp[0] = r.mo[0];
            hP[c].wamp[1] = r.mo[1];
            hP[c].wamp[2] = r.mo[2];
            hP[c].womega = r.mo[3];
            hP[c].wroll = r.mo[4];
            hP[c].wpivot[0] = r.mo[5];
            hP[c].wpivot[1] = r.mo[6];
            hP[c].wpivot[2] = r.mo[7];
            wflag_h[c] = r.fl;
            wvel_h[c] = r.wv;
            hP[c].wvel = r.wv.empty() ? 0 : 1;
        }
        RETCHK(upload_walls());
        configured = false;
        return SPHX_OK;
    }


    // c >= 0: one case into out[0]; c < 0: every case into out[0..C).
    int diagnostics(int c, sphx_diag* out) override
    {
        if (!out) return ctx->fail(SPHX_EINVAL, "NULL output");
        if (c >= C) return ctx->fail(SPHX_EINVAL, "case index out of range");
        RETCHK(ensure_layout());
        std::vector<double> r((size_t)NDIAG * C, 0.0);
        if (ntiles > 0) {
            k_diag<D, real><<<nblk(ntot), BLOCK, 0, s>>>(dP, tcase, ntiles, x[cur][0], x[cur][1], x[cur][2], st[cur],
                                                          diag_part);
            k_diag_fin<real><<<C, BLOCK, 0, s>>>(dP, diag_part, diag_out);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(r.data(), diag_out, sizeof(double) * NDIAG * C, hipMemcpyDeviceToHost, s));
        }
        RETCHK(sync_ctrl());
        for (int d = (c < 0 ? 0 : c), k = 0; d < (c < 0 ? C : c + 1); ++d, ++k) fill_diag(d, &r[(size_t)d * NDIAG], out[k]);
        return SPHX_OK;
    }

    // The same observables with the per-tile partials and the per-case sums
    // in the GPU's file-scope scratch: no allocation of any kind (device or
    // host) in the call. Needs the device layout (SPHX_ESTATE before the
    // first call that makes it) and at most SCRATCH_DOUBLES / NDIAG tiles and
    // cases together (SPHX_EINVAL beyond). Calls that overlap on one GPU share
    // its scratch and race; every value read is written by the same call.
    int diagnostics_noalloc(int c, sphx_diag* out) override
    {
        if (!out) return ctx->fail(SPHX_EINVAL, "NULL output");
        if (c >= C) return ctx->fail(SPHX_EINVAL, "case index out of range");
        if (!laid_out)
            return ctx->fail(SPHX_ESTATE, "no device layout yet (it is made by the first call that needs the "
                                          "particles, e.g. sphx_build_neighbors; this call allocates nothing)");
        const size_t need = (size_t)NDIAG * ((size_t)ntiles + (size_t)C);
        if (need > SCRATCH_DOUBLES)
            return ctx->fail(SPHX_EINVAL, "batch too large for the allocation-free diagnostics: tiles of 64 "
                                          "particle slots plus cases must not exceed 65536 (4 MiB of scratch)");
        double* base = (ctx->device >= 0 && ctx->device < SCRATCH_MAX_DEVICES) ? scratch_addr[ctx->device] : nullptr;
        if (!base) return ctx->fail(SPHX_EHIP, "device scratch address unknown");
        double* part = base;
        double* sums = base + (size_t)NDIAG * ntiles;
        constexpr int CHUNK = 32;  // cases per copy through the stack buffer
        double r[NDIAG * CHUNK];
        const int c0 = c < 0 ? 0 : c, c1 = c < 0 ? C : c + 1;
        if (ntiles > 0) {
            k_diag<D, real><<<nblk(ntot), BLOCK, 0, s>>>(dP, tcase, ntiles, x[cur][0], x[cur][1], x[cur][2], st[cur],
                                                          part);
            k_diag_fin<real><<<C, BLOCK, 0, s>>>(dP, part, sums);
            HIPCHK(hipGetLastError());
        }
        RETCHK(sync_ctrl());
        for (int d0 = c0; d0 < c1; d0 += CHUNK) {
            const int nd = std::min(CHUNK, c1 - d0);
            if (ntiles > 0) {
                HIPCHK(hipMemcpyAsync(r, sums + (size_t)d0 * NDIAG, sizeof(double) * NDIAG * nd, hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
            } else {
                for (int q = 0; q < NDIAG * nd; ++q) r[q] = 0.0;
            }
            for (int k = 0; k < nd; ++k) fill_diag(d0 + k, r + (size_t)k * NDIAG, out[d0 - c0 + k]);
        }
        return SPHX_OK;
    }

    void fill_diag(int d, const double* v, sphx_diag& o) const
    {
        {
            bool any = hP[d].nf > 0;
            o.mass = hP[d].md * hP[d].nf;
            o.momentum[0] = v[0];
            o.momentum[1] = v[1];
            o.momentum[2] = v[2];
            o.e_kin = v[3];
            o.e_pot = v[4];
            o.e_int = v[5];
            o.front = any ? v[6] : 0.0;
            o.max_drho = v[7];
            o.t = hctrl[d].t;
            o.n_substeps = hctrl[d].nsub_total;
            o.n_steps = hctrl[d].steps_done;
        }
    }

    template <typename F>
    int time_launches(int reps, double* ms, F launch)
    {
        hipEvent_t ev[2];
        HIPCHK(hipEventCreate(&ev[0]));
        HIPCHK(hipEventCreate(&ev[1]));
        float t = 0.f;
        HIPCHK(hipEventRecord(ev[0], s));
        for (int r = 0; r < reps; ++r) launch();
        HIPCHK(hipEventRecord(ev[1], s));
        HIPCHK(hipEventSynchronize(ev[1]));
        HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        HIPCHK(hipGetLastError());
        *ms = (double)t / reps;
        return SPHX_OK;
    }

    template <int T>
    int profile_t(int reps, double* ms)
    {
        const int nb = pair_blocks();
        const int a = cur;
        RETCHK(time_launches(reps, &ms[0], [&] {
            by_motion([&](auto mc) {
                constexpr int TP = pressure_lanes<T>();
                k_pressure<D, real, TP, decltype(mc)::value, T><<<pair_blocks_t<TP>(), pair_threads<TP>(), 0, s>>>(
                    dP, tcase, ctrl, geo[a], wgeo, wnrm, nbr, ncnt, wnb, wcnt, st[a], dr3[a], hf, nullptr, 0, 0,
                    vslot, avt_arg(), wmot_arg(), wvg_arg());
            });
        }));
        RETCHK(time_launches(reps, &ms[1], [&] {
            by_motion([&](auto mc) {
                k_density<D, real, T, decltype(mc)::value><<<nb, pair_threads<T>(), 0, s>>>(
                    dP, tcase, ctrl, 1, geo[a], wgeo, wnrm, nbr, ncnt, wnb, wcnt, hf, st[a], dr3[a], x[a][0],
                    x[a][1], x[a][2], nullptr, vslot, 0, avt_arg(), wmot_arg(), wvg_arg(), 0, nullptr, nullptr, nullptr,
                    nullptr);
            });
        }));
        // the list build is idempotent on the current set
        RETCHK(time_launches(reps, &ms[2], [&] { launch_neighbors<T>(1, a); }));
        RETCHK(time_launches(reps, &ms[3], [&] {
            k_reinit<D, real, T><<<nb, pair_threads<T>(), 0, s>>>(dP, tcase, ctrl, 0, geo[a], wgeo, nbr, ncnt, wnb, wcnt, st[a]);
        }));
        return SPHX_OK;
    }

    // Per-launch device time of the hot kernels on the current state of
    // every case (each case one sub-step of its own dt_ac); the state and the
    // clocks are restored afterwards.
    int profile(int32_t reps, double* ms) override
    {
        if (!configured) return ctx->fail(SPHX_ESTATE, "no neighbour configuration");
        if (reps < 1 || !ms) return ctx->fail(SPHX_EINVAL, "bad profile arguments");
        RETCHK(sync_ctrl());
        std::vector<Ctrl> saved(hctrl, hctrl + C);
        RETCHK(backup_state());
        for (int c = 0; c < C; ++c) {
            double dt_ac = hP[c].cfl_ac_h / (hP[c].c0d + hctrl[c].vmax);
            hctrl[c].ss[0] = SubState{0.0, dt_ac, 0, 1, 0, 0};
            hctrl[c].midstep = 0;
            hctrl[c].err = 0;
        }
        RETCHK(push_ctrl());
        int rc_t = SPHX_OK;
        by_lanes([&](auto t) { rc_t = profile_t<decltype(t)::value>(reps, ms); });
        RETCHK(rc_t);
        RETCHK(sync_ctrl());
        int rc = first_error();
        RETCHK(restore_state(saved));
        // the |v| slots the profiled launches filled
        HIPCHK(hipMemsetAsync(vslot, 0, sizeof(unsigned long long) * 2 * VSLOTS * C, s));
        HIPCHK(hipStreamSynchronize(s));
        return rc;
    }

    int counts(int c, int64_t* out) override
    {
        if (!out) return ctx->fail(SPHX_EINVAL, "NULL output");
        if (c >= C) return ctx->fail(SPHX_EINVAL, "case index out of range");
        RETCHK(ensure_layout());
        out[0] = out[1] = out[2] = out[3] = 0;
        for (int d = 0; d < C; ++d)
            if (c < 0 || d == c) {
                out[0] += hP[d].nf;
                out[1] += hP[d].nw;
            }
        if (!configured || ntot == 0) return SPHX_OK;
        std::vector<int32_t> a(ntot), b(ntot);
        HIPCHK(hipMemcpyAsync(a.data(), ncnt, sizeof(int32_t) * ntot, hipMemcpyDeviceToHost, s));
        HIPCHK(hipMemcpyAsync(b.data(), wcnt, sizeof(int32_t) * ntot, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int d = 0; d < C; ++d) {
            if (c >= 0 && d != c) continue;
            for (int i = hP[d].fbase; i < hP[d].fbase + hP[d].nf; ++i) {
                out[2] += a[i];
                out[3] += b[i];
            }
        }
        return SPHX_OK;
    }

    // Pick the lanes per particle of the pair kernels (2, 4 or 8 in 2D; 4, 8
    // or 16 in 3D) by timing
    // the pressure and density relaxations of every case with each; the lists
    // are rebuilt in the chosen layout (the same lists; sums are combined in
    // a different order, so results change at rounding level).
    int autotune(int32_t reps, int32_t* lanes, double* times) override
    {
        if (!configured) return ctx->fail(SPHX_ESTATE, "no neighbour configuration");
        if (reps < 1) return ctx->fail(SPHX_EINVAL, "bad repetition count");
        const int cand[3] = {D == 2 ? 2 : 4, D == 2 ? 4 : 8, D == 2 ? 8 : 16};
        double tk[3] = {1e300, 1e300, 1e300};
        // each candidate timed twice, in forward then in reverse order (the
        // first launches after a rebuild run on a cold GPU); its best counts
        for (int pass = 0; pass < 2; ++pass)
            for (int kk = 0; kk < 3; ++kk) {
                const int k = pass == 0 ? kk : 2 - kk;
                ln = cand[k];
                drop_graphs();
                RETCHK(build_neighbors());
                double ms[4];
                RETCHK(profile(reps, ms));
                tk[k] = std::fmin(tk[k], ms[0] + ms[1]);
            }
        double best = 1e300;
        int best_ln = cand[0];
        for (int k = 0; k < 3; ++k) {
            if (times) times[k] = tk[k];
            if (tk[k] < best) {
                best = tk[k];
                best_ln = cand[k];
            }
        }
        ln = best_ln;
        drop_graphs();
        RETCHK(build_neighbors());
        if (lanes) *lanes = ln;
        return SPHX_OK;
    }

    // Set the lanes per particle of the pair kernels; an existing
    // configuration is rebuilt in the new list layout (the same lists).
    int set_lanes(int32_t lanes) override
    {
        const bool ok = D == 2 ? (lanes == 2 || lanes == 4 || lanes == 8) : (lanes == 4 || lanes == 8 || lanes == 16);
        if (!ok) return ctx->fail(SPHX_EINVAL, "lanes per particle: 2, 4 or 8 in 2D; 4, 8 or 16 in 3D");
        if (lanes == ln) return SPHX_OK;
        HIPCHK(hipStreamSynchronize(s));
        ln = lanes;
        drop_graphs();
        if (configured) RETCHK(build_neighbors());
        return SPHX_OK;
    }

    // Replace case c's physical parameters; its cell grid must stay the same
    // (same box, periodicity and cell size), its particles stay.
    int set_params_case(int c, const sphx_params* q) override
    {
        RETCHK(check_case(c));
        if (!q || q->dim != D || q->precision != ctx->prm[c].precision || !(q->dp > 0) || !(q->h > 0) ||
            !(q->rho0 > 0) || !(q->c0 > 0) || !(q->u_ref > 0) || !(q->cfl_ad > 0) || !(q->cfl_ac > 0))
            return ctx->fail(SPHX_EINVAL, "bad parameters");
        const KP<real> old = hP[c];
        const sphx_params oldq = ctx->prm[c];
        ctx->prm[c] = *q;
        int rc = init_case(c, old.cbase);
        bool same = rc == SPHX_OK && hP[c].ncell == old.ncell;
        for (int k = 0; k < 3 && same; ++k) same = hP[c].n[k] == old.n[k] && hP[c].Ld[k] == old.Ld[k] &&
                                                   hP[c].lo[k] == old.lo[k] && hP[c].periodic[k] == old.periodic[k];
        if (!same) {
            hP[c] = old;
            ctx->prm[c] = oldq;
            return rc != SPHX_OK ? rc : ctx->fail(SPHX_EINVAL, case_tag(c) + "the cell grid would change");
        }
        hP[c].fbase = old.fbase;
        hP[c].nf = old.nf;
        hP[c].fcap = old.fcap;
        hP[c].wbase = old.wbase;
        hP[c].nw = old.nw;
        hP[c].wmove = old.wmove;
        hP[c].wvel = old.wvel;
        for (int k = 0; k < 3; ++k) {
            hP[c].wamp[k] = old.wamp[k];
            hP[c].wpivot[k] = old.wpivot[k];
        }
        hP[c].womega = old.womega;
        hP[c].wroll = old.wroll;
        RETCHK(upload_params());
        drop_graphs();  // the queue may gain or lose the advection-step forces
        configured = false;
        return SPHX_OK;
    }

    // ------------------------------------------------------------------
    // Message-passing surrogate (2D). Node rows are the fluid slots, edge rows
    // the CSR of each particle's inner then contact list entries.
    struct Gnn {
        GnnLayout L;
        bool ready = false;
        long long step = 0;
        long long gen = -1;       // configuration generation of the last forward
        float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
        uint16_t *wt = nullptr, *wn = nullptr;
        int Ncap = 0;
        long long Ecap = 0;
        bool Ecap_train = false, Ncap_train = false;
        std::vector<void*> fixed, nodes, edges;
        int32_t *ecount = nullptr, *eoff = nullptr, *bsumN = nullptr, *edst = nullptr, *erev = nullptr,
                *esrc = nullptr;
        bool fused = true;  // inference forward with the fused layer kernel (else edge activations in HBM)
        float *F = nullptr, *X[3] = {}, *Hs = nullptr, *Z[3] = {}, *P = nullptr, *Q = nullptr, *D1 = nullptr,
              *Y = nullptr, *T = nullptr, *dY = nullptr;
        float *dH = nullptr, *dZ = nullptr, *dA = nullptr, *dPb = nullptr, *dQb = nullptr, *wsum = nullptr;
        float *G = nullptr, *E0 = nullptr, *R = nullptr, *pre[3] = {}, *dM = nullptr, *dE0 = nullptr;
        float *part = nullptr, *bpart = nullptr;
        double *lpart = nullptr, *dtc = nullptr, *tmax = nullptr;
        int32_t* accept = nullptr;
        std::vector<long long> target_gen;   // configuration generation each case's target was set on
        long long E = 0;
    } gn;
    long long conf_gen = 0;      // incremented by every configuration update
    static constexpr int PART_BLOCKS = 1024;

    int gnn_fixed_alloc()
    {
        if (gn.p) return SPHX_OK;
        auto& A = gn.fixed;
        const int np = gn.L.total;
        RETCHK(dalloc(A, gn.p, np));
        RETCHK(dalloc(A, gn.g, np));
        RETCHK(dalloc(A, gn.m, np));
        RETCHK(dalloc(A, gn.v, np));
        RETCHK(dalloc(A, gn.wt, gn.L.ptotal));
        RETCHK(dalloc(A, gn.wn, gn.L.ptotal));
        RETCHK(dalloc(A, gn.part, (size_t)PART_BLOCKS * 128 * gnn::HID));
        RETCHK(dalloc(A, gn.bpart, (size_t)PART_BLOCKS * gnn::HID));
        RETCHK(dalloc(A, gn.dtc, C));
        RETCHK(dalloc(A, gn.accept, C));
        HIPCHK(hipMemsetAsync(gn.g, 0, sizeof(float) * np, s));
        return SPHX_OK;
    }

    // Node buffers for N slots (the training ones included: they are small).
    int gnn_nodes(bool)
    {
        const bool train = true;
        const int N = std::max(ntot, TILE);
        if (gn.Ncap >= N && gn.Ncap_train) return SPHX_OK;
        HIPCHK(hipStreamSynchronize(s));
        free_list(gn.nodes);
        auto& A = gn.nodes;
        const size_t n64 = (size_t)N * gnn::HID;
        RETCHK(dalloc(A, gn.ecount, N));
        RETCHK(dalloc(A, gn.eoff, N + 1));
        RETCHK(dalloc(A, gn.bsumN, (N + SCAN_TILE - 1) / SCAN_TILE + 1));
        RETCHK(dalloc(A, gn.F, (size_t)N * gnn::FPAD));
        for (int l = 0; l < 3; ++l) {
            RETCHK(dalloc(A, gn.X[l], 2 * n64));
            RETCHK(dalloc(A, gn.Z[l], n64));
        }
        RETCHK(dalloc(A, gn.Hs, n64));
        RETCHK(dalloc(A, gn.P, n64));
        RETCHK(dalloc(A, gn.Q, n64));
        RETCHK(dalloc(A, gn.D1, n64));
        RETCHK(dalloc(A, gn.Y, (size_t)N * gnn::NOUT));
        RETCHK(dalloc(A, gn.T, (size_t)N * gnn::NOUT));
        RETCHK(dalloc(A, gn.dY, (size_t)N * gnn::NOUT));
        RETCHK(dalloc(A, gn.lpart, nblk(N)));
        RETCHK(dalloc(A, gn.tmax, N / TILE + 1));
        if (train) {
            RETCHK(dalloc(A, gn.dH, n64));
            RETCHK(dalloc(A, gn.dZ, n64));
            RETCHK(dalloc(A, gn.dA, n64));
            RETCHK(dalloc(A, gn.dPb, n64));
            RETCHK(dalloc(A, gn.dQb, n64));
            RETCHK(dalloc(A, gn.wsum, n64));
        }
        HIPCHK(hipMemsetAsync(gn.T, 0, sizeof(float) * (size_t)N * gnn::NOUT, s));
        gn.Ncap = N;
        gn.Ncap_train = train;
        gn.target_gen.assign(C, -1);
        gn.gen = -1;
        return SPHX_OK;
    }

    int gnn_edges_alloc(long long E, bool train)
    {
        E = std::max(E, 1LL);
        if (gn.Ecap >= E && (!train || gn.Ecap_train)) return SPHX_OK;
        HIPCHK(hipStreamSynchronize(s));
        free_list(gn.edges);
        auto& A = gn.edges;
        const long long cap = E + E / 8 + 1024;
        const size_t e64 = (size_t)cap * gnn::HID;
        RETCHK(dalloc(A, gn.edst, cap));
        RETCHK(dalloc(A, gn.erev, cap));
        RETCHK(dalloc(A, gn.esrc, cap));
        RETCHK(dalloc(A, gn.G, (size_t)cap * gnn::FPAD));
        RETCHK(dalloc(A, gn.E0, e64));
        RETCHK(dalloc(A, gn.R, e64));
        if (train) {
            for (int l = 0; l < 3; ++l) RETCHK(dalloc(A, gn.pre[l], e64));
            RETCHK(dalloc(A, gn.dM, e64));
            RETCHK(dalloc(A, gn.dE0, e64));
        } else {
            for (int l = 0; l < 3; ++l) gn.pre[l] = nullptr;
        }
        gn.Ecap = cap;
        gn.Ecap_train = train;
        return SPHX_OK;
    }

    int gnn_check_ready()
    {
        if (D != 2) return ctx->fail(SPHX_EINVAL, "the surrogate is two-dimensional");
        if (any_move() || any_wvel()) return ctx->fail(SPHX_EINVAL, "the surrogate models static walls only");
        if (!gn.ready) return ctx->fail(SPHX_ESTATE, "surrogate parameters not set");
        if (!configured) return ctx->fail(SPHX_ESTATE, "no neighbour configuration");
        return SPHX_OK;
    }

    int gnn_pack()
    {
        auto pack = [&](int K, int off, int pk) {
            gnn::k_pack_w<<<(K * gnn::HID + 255) / 256, 256, 0, s>>>(K, gn.p + off, gn.wt + pk, gn.wn + pk);
        };
        pack(32, gn.L.Wn, gn.L.pWn);
        pack(32, gn.L.We, gn.L.pWe);
        for (int l = 0; l < 3; ++l) {
            pack(64, gn.L.Wa[l], gn.L.pWa[l]);
            pack(64, gn.L.Wb[l], gn.L.pWb[l]);
            pack(64, gn.L.Wc[l], gn.L.pWc[l]);
            pack(128, gn.L.Wu[l], gn.L.pWu[l]);
        }
        pack(64, gn.L.Wo1, gn.L.pWo1);
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    int gnn_set_params(const float* p, int64_t n) override
    {
        if (D != 2) return ctx->fail(SPHX_EINVAL, "the surrogate is two-dimensional");
        if (!p || n != gn.L.total) return ctx->fail(SPHX_EINVAL, "parameter array of the wrong size");
        RETCHK(gnn_fixed_alloc());
        HIPCHK(hipMemcpyAsync(gn.p, p, sizeof(float) * n, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemsetAsync(gn.m, 0, sizeof(float) * n, s));
        HIPCHK(hipMemsetAsync(gn.v, 0, sizeof(float) * n, s));
        HIPCHK(hipMemsetAsync(gn.g, 0, sizeof(float) * n, s));
        RETCHK(gnn_pack());
        HIPCHK(hipStreamSynchronize(s));
        gn.step = 0;
        gn.ready = true;
        gn.gen = -1;
        return SPHX_OK;
    }

    // which: 0 parameters, 1 gradient of the last training step
    int gnn_get(int which, float* p, int64_t n) override
    {
        if (D != 2) return ctx->fail(SPHX_EINVAL, "the surrogate is two-dimensional");
        if (!gn.ready) return ctx->fail(SPHX_ESTATE, "surrogate parameters not set");
        if (!p || n != gn.L.total) return ctx->fail(SPHX_EINVAL, "parameter array of the wrong size");
        HIPCHK(hipMemcpyAsync(p, which == 0 ? gn.p : gn.g, sizeof(float) * n, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return SPHX_OK;
    }

    // The CSR graph and the features of the current configuration (with
    // `compact`: the edge features alone per row, source indices, no reverse
    // edges, for the fused inference layer).
    int gnn_graph(bool train, bool compact = false)
    {
        RETCHK(gnn_nodes(train));
        const int N = ntot;
        gnn::k_gnn_count<real><<<nblk(N), BLOCK, 0, s>>>(dP, tcase, ntiles, ncnt, wcnt, gn.ecount);
        const int nb = (N + SCAN_TILE - 1) / SCAN_TILE;
        k_scan_tiles<<<nb, BLOCK, 0, s>>>(gn.ecount, gn.eoff, gn.bsumN, N);
        k_scan_top<<<1, BLOCK, 0, s>>>(gn.bsumN, nb);
        k_scan_add<<<nb, BLOCK, 0, s>>>(gn.eoff, gn.bsumN, N, nb);
        HIPCHK(hipGetLastError());
        int32_t etot = 0;
        HIPCHK(hipMemcpyAsync(&etot, gn.eoff + N, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        gn.E = etot;
        RETCHK(gnn_edges_alloc(gn.E, train));
        if constexpr (D == 2) {
            by_lanes([&](auto t) {
                gnn::k_gnn_edges<real, decltype(t)::value><<<nblk(N), BLOCK, 0, s>>>(
                    dP, tcase, ntiles, gn.eoff, nbr, ncnt, wnb, wcnt, geo[cur], wgeo, st[cur], gn.edst,
                    compact ? nullptr : gn.erev, compact ? gn.esrc : nullptr, gn.G, compact ? gnn::EFEAT : gnn::FPAD,
                    gn.F);
            });
        }
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    template <int K, int EPI>
    void gemm(long long M, const float* A, int lda, const uint16_t* Bt, const float* bias, float* Cm, int ldc,
              float* C2 = nullptr, int ldc2 = 0)
    {
        if (M <= 0) return;
        gnn::k_gemm64<K, EPI><<<(int)((M + 63) / 64), 256, 0, s>>>((int)M, A, lda, Bt, bias, Cm, ldc, C2, ldc2);
    }

    // dW (KIN x 64) and optionally db (64) from X^T dZ over M rows.
    template <int KIN>
    void wgrad(long long M, const float* X, int ldx, const float* dZ, int ldz, float* dW, float* db)
    {
        if (M <= 0) return;
        int rows = (int)((M + PART_BLOCKS - 1) / PART_BLOCKS);
        rows = std::max(256, (rows + 31) / 32 * 32);
        const int nb = (int)((M + rows - 1) / rows);
        gnn::k_wgrad<KIN><<<nb, 256, 0, s>>>((int)M, rows, X, ldx, dZ, ldz, gn.part, gn.bpart);
        gnn::k_reduce_parts<<<(KIN * gnn::HID + 255) / 256, 256, 0, s>>>(nb, KIN * gnn::HID, gn.part, dW, 0);
        if (db) gnn::k_reduce_parts<<<1, 256, 0, s>>>(nb, gnn::HID, gn.bpart, db, 0);
    }

    void elem64(long long M, const float* src, int lds, const float* mask, int ldm, float* out, int ldo)
    {
        if (M <= 0) return;
        const long long n = M * gnn::HID;
        if (mask)
            gnn::k_relu_mask<<<(int)((n + 255) / 256), 256, 0, s>>>((int)M, src, lds, mask, ldm, out, ldo);
        else
            gnn::k_copy64<<<(int)((n + 255) / 256), 256, 0, s>>>((int)M, src, lds, out, ldo);
    }

    static constexpr int FUSED_NPW = 8;  // nodes per wavefront of the fused layer

    void fused_layer(int l)
    {
        const int N = ntot;
        const int per_block = 4 * FUSED_NPW;
        gnn::k_gnn_layer_fused<FUSED_NPW><<<(N + per_block - 1) / per_block, 256, 0, s>>>(
            N, gn.eoff, gn.edst, gn.esrc, gn.G, gn.wt + gn.L.pWe, gn.p + gn.L.be, gn.wt + gn.L.pWc[l], gn.P, gn.Q,
            gn.p + gn.L.qw[l], gn.X[l]);
    }

    int gnn_forward_impl(bool train)
    {
        // inference: the fused layers (E0, R and the messages stay on chip)
        if (!train && gn.fused) return gnn_forward_fused();
        RETCHK(gnn_graph(train));
        const GnnLayout& L = gn.L;
        const int N = ntot;
        const long long E = gn.E;
        float* p = gn.p;
        constexpr int H = gnn::HID;
        gemm<32, gnn::EPI_RELU>(N, gn.F, 32, gn.wt + L.pWn, p + L.bn, gn.X[0], 2 * H);
        elem64(N, gn.X[0], 2 * H, nullptr, 0, gn.Hs, H);
        gemm<32, gnn::EPI_RELU>(E, gn.G, 32, gn.wt + L.pWe, p + L.be, gn.E0, H);
        for (int l = 0; l < 3; ++l) {
            gemm<64, gnn::EPI_STORE>(N, gn.X[l], 2 * H, gn.wt + L.pWa[l], p + L.bm[l], gn.P, H);
            gemm<64, gnn::EPI_STORE>(N, gn.X[l], 2 * H, gn.wt + L.pWb[l], nullptr, gn.Q, H);
            gemm<64, gnn::EPI_STORE>(E, gn.E0, H, gn.wt + L.pWc[l], nullptr, gn.R, H);
            gnn::k_gnn_msg<<<(N + 3) / 4, 256, 0, s>>>(N, gn.eoff, gn.edst, gn.P, gn.Q, gn.R, p + L.qw[l],
                                                       train ? gn.pre[l] : nullptr, gn.X[l]);
            gemm<128, gnn::EPI_RESID>(N, gn.X[l], 2 * H, gn.wt + L.pWu[l], p + L.bu[l], gn.Hs, H, gn.Z[l], H);
            if (l < 2) elem64(N, gn.Hs, H, nullptr, 0, gn.X[l + 1], 2 * H);
        }
        gemm<64, gnn::EPI_RELU>(N, gn.Hs, H, gn.wt + L.pWo1, p + L.bo1, gn.D1, H);
        gnn::k_gnn_out<<<nblk(N), BLOCK, 0, s>>>(N, gn.D1, p + L.Wo2, p + L.bo2, gn.Y);
        HIPCHK(hipGetLastError());
        gn.gen = conf_gen;
        return SPHX_OK;
    }

    int gnn_forward_fused()
    {
        RETCHK(gnn_graph(false, true));
        const GnnLayout& L = gn.L;
        const int N = ntot;
        float* p = gn.p;
        constexpr int H = gnn::HID;
        gemm<32, gnn::EPI_RELU>(N, gn.F, 32, gn.wt + L.pWn, p + L.bn, gn.X[0], 2 * H);
        elem64(N, gn.X[0], 2 * H, nullptr, 0, gn.Hs, H);
        for (int l = 0; l < 3; ++l) {
            gemm<64, gnn::EPI_STORE>(N, gn.X[l], 2 * H, gn.wt + L.pWa[l], p + L.bm[l], gn.P, H);
            gemm<64, gnn::EPI_STORE>(N, gn.X[l], 2 * H, gn.wt + L.pWb[l], nullptr, gn.Q, H);
            fused_layer(l);
            gemm<128, gnn::EPI_RESID>(N, gn.X[l], 2 * H, gn.wt + L.pWu[l], p + L.bu[l], gn.Hs, H, gn.Z[l], H);
            if (l < 2) elem64(N, gn.Hs, H, nullptr, 0, gn.X[l + 1], 2 * H);
        }
        gemm<64, gnn::EPI_RELU>(N, gn.Hs, H, gn.wt + L.pWo1, p + L.bo1, gn.D1, H);
        gnn::k_gnn_out<<<nblk(N), BLOCK, 0, s>>>(N, gn.D1, p + L.Wo2, p + L.bo2, gn.Y);
        HIPCHK(hipGetLastError());
        gn.gen = conf_gen;
        return SPHX_OK;
    }

    int gnn_backward_impl()
    {
        const GnnLayout& L = gn.L;
        const int N = ntot;
        const long long E = gn.E;
        float *p = gn.p, *g = gn.g;
        constexpr int H = gnn::HID;
        // decoder
        {
            const int rows = std::max(256, (N + PART_BLOCKS - 1) / PART_BLOCKS);
            const int nb = (N + rows - 1) / rows;
            gnn::k_gnn_out_wgrad<<<nb, 256, 0, s>>>(N, rows, gn.D1, gn.dY, gn.part);
            gnn::k_reduce_parts<<<1, 256, 0, s>>>(nb, H * 3 + 3, gn.part, g + L.Wo2, 0);
            const long long n = (long long)N * H;
            gnn::k_gnn_out_bwd<<<(int)((n + 255) / 256), 256, 0, s>>>(N, gn.D1, gn.dY, p + L.Wo2, gn.dZ);
        }
        wgrad<64>(N, gn.Hs, H, gn.dZ, H, g + L.Wo1, g + L.bo1);
        gemm<64, gnn::EPI_STORE>(N, gn.dZ, H, gn.wn + L.pWo1, nullptr, gn.dH, H);
        for (int l = 2; l >= 0; --l) {
            elem64(N, gn.dH, H, gn.Z[l], H, gn.dZ, H);
            wgrad<128>(N, gn.X[l], 2 * H, gn.dZ, H, g + L.Wu[l], g + L.bu[l]);
            gemm<64, gnn::EPI_ACCUM>(N, gn.dZ, H, gn.wn + L.pWu[l], nullptr, gn.dH, H);
            gemm<64, gnn::EPI_STORE>(N, gn.dZ, H, gn.wn + L.pWu[l] + 64 * H, nullptr, gn.dA, H);
            gnn::k_gnn_msg_bwd<<<(N + 3) / 4, 256, 0, s>>>(N, gn.eoff, gn.edst, gn.pre[l], gn.dA, H, gn.dM, gn.dPb,
                                                           gn.wsum);
            gnn::k_gnn_dq<<<(N + 3) / 4, 256, 0, s>>>(N, gn.eoff, gn.edst, gn.erev, gn.dM, gn.dQb);
            {
                const int rows = std::max(256, (N + PART_BLOCKS - 1) / PART_BLOCKS);
                const int nb = (N + rows - 1) / rows;
                gnn::k_colsum64<<<nb, 64, 0, s>>>(N, rows, gn.wsum, H, gn.bpart);
                gnn::k_reduce_parts<<<1, 256, 0, s>>>(nb, H, gn.bpart, g + L.qw[l], 0);
            }
            wgrad<64>(N, gn.X[l], 2 * H, gn.dPb, H, g + L.Wa[l], g + L.bm[l]);
            wgrad<64>(N, gn.X[l], 2 * H, gn.dQb, H, g + L.Wb[l], nullptr);
            wgrad<64>(E, gn.E0, H, gn.dM, H, g + L.Wc[l], nullptr);
            gemm<64, gnn::EPI_ACCUM>(N, gn.dPb, H, gn.wn + L.pWa[l], nullptr, gn.dH, H);
            gemm<64, gnn::EPI_ACCUM>(N, gn.dQb, H, gn.wn + L.pWb[l], nullptr, gn.dH, H);
            if (l == 2) gemm<64, gnn::EPI_STORE>(E, gn.dM, H, gn.wn + L.pWc[l], nullptr, gn.dE0, H);
            else gemm<64, gnn::EPI_ACCUM>(E, gn.dM, H, gn.wn + L.pWc[l], nullptr, gn.dE0, H);
        }
        // encoders (dM is free again: it takes dZe)
        elem64(E, gn.dE0, H, gn.E0, H, gn.dM, H);
        wgrad<32>(E, gn.G, 32, gn.dM, H, g + L.We, g + L.be);
        elem64(N, gn.dH, H, gn.X[0], 2 * H, gn.dZ, H);
        wgrad<32>(N, gn.F, 32, gn.dZ, H, g + L.Wn, g + L.bn);
        HIPCHK(hipGetLastError());
        return SPHX_OK;
    }

    int gnn_forward() override
    {
        RETCHK(gnn_check_ready());
        RETCHK(gnn_forward_impl(false));
        HIPCHK(hipStreamSynchronize(s));
        return SPHX_OK;
    }

    int gnn_get_output(int c, double* out) override
    {
        RETCHK(check_case(c));
        if (!out) return ctx->fail(SPHX_EINVAL, "NULL output");
        if (gn.gen != conf_gen || gn.gen < 0) return ctx->fail(SPHX_ESTATE, "no surrogate output for this configuration");
        const KP<real>& P = hP[c];
        if (P.nf == 0) return SPHX_OK;
        k_unsort_vec<float><<<nblk(P.nf), BLOCK, 0, s>>>(P.fbase, P.nf, gnn::NOUT, id[cur], gn.Y, outbuf);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(out, outbuf, sizeof(double) * (size_t)P.nf * gnn::NOUT, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        return SPHX_OK;
    }

    int gnn_set_target(int c, const double* t) override
    {
        RETCHK(check_case(c));
        if (D != 2) return ctx->fail(SPHX_EINVAL, "the surrogate is two-dimensional");
        if (!t) return ctx->fail(SPHX_EINVAL, "NULL target");
        if (!configured) return ctx->fail(SPHX_ESTATE, "no neighbour configuration");
        RETCHK(gnn_nodes(false));
        const KP<real>& P = hP[c];
        if (P.nf > 0) {
            RETCHK(ensure_stage((size_t)P.nf * gnn::NOUT));
            HIPCHK(hipMemcpyAsync(stage, t, sizeof(double) * (size_t)P.nf * gnn::NOUT, hipMemcpyHostToDevice, s));
            gnn::k_gnn_load_target<real><<<nblk(P.nf), BLOCK, 0, s>>>(dP, c, id[cur], stage, gn.T);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(s));
        }
        gn.target_gen[c] = conf_gen;
        return SPHX_OK;
    }

    int gnn_train_step(double lr, double* loss) override
    {
        RETCHK(gnn_check_ready());
        RETCHK(gnn_nodes(true));
        for (int c = 0; c < C; ++c)
            if (gn.target_gen[c] != conf_gen)
                return ctx->fail(SPHX_ESTATE, case_tag(c) + "no training target set on the current configuration");
        long long count = 0;
        for (int c = 0; c < C; ++c) count += hP[c].nf;
        RETCHK(gnn_forward_impl(true));
        const int nbl = nblk(ntot);
        gnn::k_gnn_loss<real><<<nbl, 256, 0, s>>>(dP, tcase, ntiles, 1.0 / (3.0 * (double)count), gn.Y, gn.T, gn.dY,
                                                  gn.lpart);
        HIPCHK(hipGetLastError());
        RETCHK(gnn_backward_impl());
        gn.step += 1;
        const double b1 = 0.9, b2 = 0.999;
        const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)gn.step)));
        const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)gn.step)));
        gnn::k_adam<<<(gn.L.total + 255) / 256, 256, 0, s>>>(gn.L.total, gn.p, gn.g, gn.m, gn.v, (float)lr, (float)b1,
                                                            (float)b2, 1e-8f, c1, c2);
        HIPCHK(hipGetLastError());
        RETCHK(gnn_pack());
        std::vector<double> lp(nbl);
        HIPCHK(hipMemcpyAsync(lp.data(), gn.lpart, sizeof(double) * nbl, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double sum = 0.0;
        for (double v : lp) sum += v;
        if (loss) *loss = sum / (3.0 * (double)count);
        gn.gen = -1;  // the outputs belong to the parameters before the step
        return SPHX_OK;
    }

    // Per-launch device time of the surrogate's kernels on the current
    // configuration: ms[0] edge product R = E0 Wc, ms[1] message sums (one
    // layer), ms[2] node update product [H | A] Wu, ms[3] a whole forward pass
    // (graph and features included); sizes[0] nodes, sizes[1] edges.
    int gnn_profile(int32_t reps, double* ms, int64_t* sizes) override
    {
        RETCHK(gnn_check_ready());
        if (reps < 1 || !ms) return ctx->fail(SPHX_EINVAL, "bad profile arguments");
        const GnnLayout& L = gn.L;
        const int N = ntot;
        constexpr int H = gnn::HID;
        float* p = gn.p;
        auto whole = [&](bool fused, double* out) {
            const bool keep = gn.fused;
            gn.fused = fused;
            hipEvent_t ev[2];
            HIPCHK(hipEventCreate(&ev[0]));
            HIPCHK(hipEventCreate(&ev[1]));
            HIPCHK(hipEventRecord(ev[0], s));
            int rc = SPHX_OK;
            for (int r = 0; r < reps && rc == SPHX_OK; ++r) rc = gnn_forward_impl(false);
            HIPCHK(hipEventRecord(ev[1], s));
            HIPCHK(hipEventSynchronize(ev[1]));
            float t = 0.f;
            HIPCHK(hipEventElapsedTime(&t, ev[0], ev[1]));
            (void)hipEventDestroy(ev[0]);
            (void)hipEventDestroy(ev[1]);
            gn.fused = keep;
            *out = (double)t / reps;
            return rc;
        };
        // the unfused forward (edge activations and products through HBM)
        RETCHK(whole(false, &ms[4]));
        const long long E = gn.E;
        RETCHK(time_launches(reps, &ms[5], [&] { gemm<64, gnn::EPI_STORE>(E, gn.E0, H, gn.wt + L.pWc[0], nullptr, gn.R, H); }));
        RETCHK(time_launches(reps, &ms[6], [&] {
            gnn::k_gnn_msg<<<(N + 3) / 4, 256, 0, s>>>(N, gn.eoff, gn.edst, gn.P, gn.Q, gn.R, p + L.qw[0], nullptr,
                                                       gn.X[0]);
        }));
        // the fused forward (the default)
        RETCHK(whole(true, &ms[3]));
        RETCHK(time_launches(reps, &ms[0], [&] { fused_layer(0); }));
        RETCHK(time_launches(reps, &ms[1], [&] {
            if constexpr (D == 2) {
                by_lanes([&](auto t) {
                    gnn::k_gnn_edges<real, decltype(t)::value><<<nblk(N), BLOCK, 0, s>>>(
                        dP, tcase, ntiles, gn.eoff, nbr, ncnt, wnb, wcnt, geo[cur], wgeo, st[cur], gn.edst, nullptr,
                        gn.esrc, gn.G, gnn::EFEAT, gn.F);
                });
            }
        }));
        RETCHK(time_launches(reps, &ms[2], [&] {
            gemm<128, gnn::EPI_STORE>(N, gn.X[0], 2 * H, gn.wt + L.pWu[0], p + L.bu[0], gn.Z[0], H);
        }));
        if (sizes) {
            sizes[0] = N;
            sizes[1] = E;
        }
        return SPHX_OK;
    }

    // Surrogate windows: each predicts every case's mean rates over the next
    // two advection steps (dt = 2 dt_ad from the current |v|max) and applies
    // them where the predicted density stays within max_drho of rho0 (and,
    // with plain_every > 0, except every plain_every-th window); the other
    // cases take the two steps with the plain scheme.
    int surrogate_advance(int32_t windows, double max_drho, int32_t plain_every, int64_t* n_fallback,
                          int64_t* n_surrogate) override
    {
        if (D != 2) return ctx->fail(SPHX_EINVAL, "the surrogate is two-dimensional");
        if (any_move() || any_wvel()) return ctx->fail(SPHX_EINVAL, "the surrogate models static walls only");
        if (!gn.ready) return ctx->fail(SPHX_ESTATE, "surrogate parameters not set");
        if (windows < 0) return ctx->fail(SPHX_EINVAL, "negative window count");
        RETCHK(all_have_fluid());
        if (!configured) RETCHK(build_neighbors());
        long long nfb = 0, nsu = 0;
        std::vector<double> dtc(C);
        std::vector<int32_t> acc(C);
        std::vector<double> tm;
        for (int w = 0; w < windows; ++w) {
            RETCHK(sync_ctrl());
            const bool plain_turn = plain_every > 0 && (w % plain_every) == plain_every - 1;
            if (plain_turn) {
                // a plain window for every case: no prediction needed; a run
                // of consecutive plain windows (every window, with
                // plain_every 1) goes to the device as one advance, which
                // gives the same bits as window by window
                int k = 1;
                if (plain_every == 1) k = windows - w;
                std::vector<long long> steps(C, 2LL * k);
                for (int c = 0; c < C; ++c) nfb += hctrl[c].err ? 0 : k;
                int rc = advance_cases(steps, std::numeric_limits<double>::infinity(), nullptr, nullptr);
                if (rc != SPHX_OK && rc != SPHX_EESCAPE && rc != SPHX_ENAN && rc != SPHX_EOVERFLOW) return rc;
                w += k - 1;
                continue;
            }
            RETCHK(gnn_forward_impl(false));
            for (int c = 0; c < C; ++c) {
                double dt_ad = hP[c].cfl_ad_h / std::fmax(hctrl[c].vmax, hP[c].u_ref);
                if (hP[c].visc_dt > 0.0) dt_ad = std::fmin(dt_ad, hP[c].visc_dt);
                dtc[c] = 2.0 * dt_ad;
            }
            HIPCHK(hipMemcpyAsync(gn.dtc, dtc.data(), sizeof(double) * C, hipMemcpyHostToDevice, s));
            gnn::k_gnn_check<real><<<nblk(ntot), BLOCK, 0, s>>>(dP, tcase, ntiles, gn.dtc, gn.Y, st[cur], gn.tmax);
            HIPCHK(hipGetLastError());
            tm.resize(std::max(ntiles, 1));
            HIPCHK(hipMemcpyAsync(tm.data(), gn.tmax, sizeof(double) * ntiles, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            bool any_acc = false, any_rej = false;
            for (int c = 0; c < C; ++c) {
                double mx = 0.0;
                for (int t = hP[c].fbase / TILE; t < (hP[c].fbase + hP[c].fcap) / TILE; ++t) mx = std::fmax(mx, tm[t]);
                acc[c] = !hctrl[c].err && mx <= max_drho;
                any_acc |= acc[c] != 0;
                any_rej |= !acc[c] && !hctrl[c].err;
            }
            if (any_acc) {
                HIPCHK(hipMemcpyAsync(gn.accept, acc.data(), sizeof(int32_t) * C, hipMemcpyHostToDevice, s));
                gnn::k_gnn_apply<real><<<nblk(ntot), BLOCK, 0, s>>>(dP, tcase, ntiles, gn.dtc, gn.accept, gn.Y,
                                                                     x[cur][0], x[cur][1], st[cur]);
                HIPCHK(hipGetLastError());
                for (int c = 0; c < C; ++c) {
                    hctrl[c].rebuild = acc[c];
                    hctrl[c].midstep = 0;
                    if (acc[c]) {
                        hctrl[c].t += dtc[c];
                        hctrl[c].steps_done += 2;
                        ++nsu;
                    }
                }
                RETCHK(push_ctrl());
                RETCHK(enqueue_rebuild(0, cur));
                cur ^= 1;
                ++conf_gen;
                k_vmax<D, real><<<nblk(ntot), BLOCK, 0, s>>>(dP, tcase, ntiles, -1, gn.accept, ctrl, st[cur]);
                k_vmax_fin<real><<<(C + 63) / 64, 64, 0, s>>>(ctrl, C, -1, gn.accept);
                HIPCHK(hipGetLastError());
                RETCHK(sync_ctrl());
            }
            if (any_rej) {
                std::vector<long long> steps(C);
                for (int c = 0; c < C; ++c) {
                    steps[c] = acc[c] ? 0 : 2;
                    nfb += acc[c] ? 0 : 1;
                }
                int rc = advance_cases(steps, std::numeric_limits<double>::infinity(), nullptr, nullptr);
                if (rc != SPHX_OK && rc != SPHX_EESCAPE && rc != SPHX_ENAN && rc != SPHX_EOVERFLOW) return rc;
            }
        }
        if (n_fallback) *n_fallback = nfb;
        if (n_surrogate) *n_surrogate = nsu;
        RETCHK(sync_ctrl());
        return first_error();
    }
};

// ---------------------------------------------------------------------
// C ABI

static int create_impl(const sphx_params* params, int32_t n, void* stream, sphx_ctx** out)
{
    if (!params || !out || n < 1) return SPHX_EINVAL;
    *out = nullptr;
    for (int c = 0; c < n; ++c) {
        const sphx_params& q = params[c];
        if ((q.dim != 2 && q.dim != 3) || (q.precision != SPHX_FP32 && q.precision != SPHX_FP64) || !(q.dp > 0) ||
            !(q.h > 0) || !(q.rho0 > 0) || !(q.c0 > 0) || !(q.u_ref > 0) || !(q.cfl_ad > 0) || !(q.cfl_ac > 0))
            return SPHX_EINVAL;
        if (q.dim != params[0].dim || q.precision != params[0].precision) return SPHX_EINVAL;
    }
    std::unique_ptr<sphx_ctx> ctx(new (std::nothrow) sphx_ctx());
    if (!ctx) return SPHX_ENOMEM;
    ctx->prm.assign(params, params + n);
    ctx->err.reserve(1024);
    {
        // the context's GPU, and its scratch address (set-up of the
        // allocation-free diagnostics, once per device)
        if (hipGetDevice(&ctx->device) != hipSuccess) return SPHX_EHIP;
        double* sp = nullptr;
        if (scratch_for_device(ctx->device, &sp) != hipSuccess) return SPHX_EHIP;
    }
    if (stream) {
        ctx->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return SPHX_EHIP;
        ctx->own_stream = true;
    }
    const sphx_params& q = params[0];
    if (q.dim == 2 && q.precision == SPHX_FP64) ctx->eng.reset(new Engine<2, double>(ctx.get(), n));
    else if (q.dim == 2) ctx->eng.reset(new Engine<2, float>(ctx.get(), n));
    else if (q.precision == SPHX_FP64) ctx->eng.reset(new Engine<3, double>(ctx.get(), n));
    else ctx->eng.reset(new Engine<3, float>(ctx.get(), n));
    int rc = ctx->eng->init();
    if (rc != SPHX_OK) {
        ctx->eng.reset();
        if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
        return rc;
    }
    *out = ctx.release();
    return SPHX_OK;
}

extern "C" {

int sphx_create(const sphx_params* params, void* stream, sphx_ctx** out) { return create_impl(params, 1, stream, out); }

int sphx_create_batch(const sphx_params* params, int32_t n_cases, void* stream, sphx_ctx** out)
{
    return create_impl(params, n_cases, stream, out);
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

int sphx_num_cases(const sphx_ctx* ctx) { return ctx ? ctx->eng->ncases() : SPHX_EINVAL; }

int sphx_set_fluid(sphx_ctx* ctx, int64_t n, const double* pos, const double* vel, const double* rho, const double* drho)
{
    ENG_CALL(set_fluid(0, n, pos, vel, rho, drho));
}

int sphx_set_fluid_case(sphx_ctx* ctx, int32_t c, int64_t n, const double* pos, const double* vel, const double* rho,
                        const double* drho)
{
    ENG_CALL(set_fluid(c, n, pos, vel, rho, drho));
}

int sphx_set_walls(sphx_ctx* ctx, int64_t n, const double* pos, const double* normal)
{
    ENG_CALL(set_walls(0, n, pos, normal));
}

int sphx_set_walls_case(sphx_ctx* ctx, int32_t c, int64_t n, const double* pos, const double* normal)
{
    ENG_CALL(set_walls(c, n, pos, normal));
}

int sphx_set_wall_motion(sphx_ctx* ctx, const sphx_wall_motion* motion, const int32_t* moving)
{
    ENG_CALL(set_wall_motion(0, motion, moving));
}

int sphx_set_wall_motion_case(sphx_ctx* ctx, int32_t c, const sphx_wall_motion* motion, const int32_t* moving)
{
    ENG_CALL(set_wall_motion(c, motion, moving));
}

int sphx_set_wall_velocity(sphx_ctx* ctx, const double* vel) { ENG_CALL(set_wall_velocity(0, vel)); }

int sphx_set_wall_velocity_case(sphx_ctx* ctx, int32_t c, const double* vel)
{
    ENG_CALL(set_wall_velocity(c, vel));
}

int sphx_save(sphx_ctx* ctx, const char* path) { ENG_CALL(save(path)); }

int sphx_load(sphx_ctx* ctx, const char* path) { ENG_CALL(load(path)); }

int sphx_set_fluid_device(sphx_ctx* ctx, int32_t c, int64_t n, const double* pos, const double* vel,
                          const double* rho, const double* drho)
{
    ENG_CALL(set_fluid_device(c, n, pos, vel, rho, drho));
}

int sphx_get_field_device(sphx_ctx* ctx, int32_t c, int field, double* out) { ENG_CALL(get_field_device(c, field, out)); }

int sphx_build_neighbors(sphx_ctx* ctx) { ENG_CALL(build_neighbors()); }

int sphx_get_neighbors(sphx_ctx* ctx, int kind, int64_t* off, int64_t* idx, int64_t cap, int64_t* n_out)
{
    if (ctx && kind != SPHX_INNER && kind != SPHX_CONTACT) return ctx->fail(SPHX_EINVAL, "bad neighbour kind");
    ENG_CALL(get_neighbors(0, kind, off, idx, cap, n_out));
}

int sphx_get_neighbors_case(sphx_ctx* ctx, int32_t c, int kind, int64_t* off, int64_t* idx, int64_t cap,
                            int64_t* n_out)
{
    if (ctx && kind != SPHX_INNER && kind != SPHX_CONTACT) return ctx->fail(SPHX_EINVAL, "bad neighbour kind");
    ENG_CALL(get_neighbors(c, kind, off, idx, cap, n_out));
}

int sphx_density_reinit(sphx_ctx* ctx) { ENG_CALL(density_reinit()); }

int sphx_time_steps(sphx_ctx* ctx, double* dt_ad, double* dt_ac) { ENG_CALL(time_steps(0, dt_ad, dt_ac)); }

int sphx_time_steps_case(sphx_ctx* ctx, int32_t c, double* dt_ad, double* dt_ac)
{
    ENG_CALL(time_steps(c, dt_ad, dt_ac));
}

int sphx_compute_rates(sphx_ctx* ctx, double dt, double* dvdt, double* drhodt)
{
    ENG_CALL(compute_rates(0, dt, dvdt, drhodt));
}

int sphx_compute_rates_case(sphx_ctx* ctx, int32_t c, double dt, double* dvdt, double* drhodt)
{
    ENG_CALL(compute_rates(c, dt, dvdt, drhodt));
}

int sphx_advance(sphx_ctx* ctx, int32_t n_steps, double t_stop, int64_t* n_substeps, double* t_out)
{
    ENG_CALL(advance(n_steps, t_stop, n_substeps, t_out));
}

int sphx_case_status(sphx_ctx* ctx, int32_t c) { ENG_CALL(case_status(c)); }

int sphx_get_field(sphx_ctx* ctx, int field, double* out) { ENG_CALL(get_field(0, field, out)); }

int sphx_get_field_case(sphx_ctx* ctx, int32_t c, int field, double* out) { ENG_CALL(get_field(c, field, out)); }

int sphx_diagnostics(sphx_ctx* ctx, sphx_diag* out) { ENG_CALL(diagnostics(0, out)); }

int sphx_diagnostics_case(sphx_ctx* ctx, int32_t c, sphx_diag* out) { ENG_CALL(diagnostics(c, out)); }

int sphx_diagnostics_noalloc(sphx_ctx* ctx, int32_t c, sphx_diag* out) { ENG_CALL(diagnostics_noalloc(c, out)); }

int sphx_profile(sphx_ctx* ctx, int32_t reps, double* ms) { ENG_CALL(profile(reps, ms)); }

int sphx_counts(sphx_ctx* ctx, int64_t* out) { ENG_CALL(counts(-1, out)); }

int sphx_counts_case(sphx_ctx* ctx, int32_t c, int64_t* out) { ENG_CALL(counts(c, out)); }

int sphx_set_lanes(sphx_ctx* ctx, int32_t lanes) { ENG_CALL(set_lanes(lanes)); }

int sphx_autotune(sphx_ctx* ctx, int32_t reps, int32_t* lanes, double* times)
{
    ENG_CALL(autotune(reps, lanes, times));
}

int sphx_set_params_case(sphx_ctx* ctx, int32_t c, const sphx_params* params) { ENG_CALL(set_params_case(c, params)); }

int64_t sphx_gnn_num_params(void) { return GnnLayout().total; }

int sphx_gnn_set_params(sphx_ctx* ctx, const float* params, int64_t n) { ENG_CALL(gnn_set_params(params, n)); }

int sphx_gnn_get_params(sphx_ctx* ctx, float* params, int64_t n) { ENG_CALL(gnn_get(0, params, n)); }

int sphx_gnn_get_grad(sphx_ctx* ctx, float* grad, int64_t n) { ENG_CALL(gnn_get(1, grad, n)); }

int sphx_gnn_forward(sphx_ctx* ctx) { ENG_CALL(gnn_forward()); }

int sphx_gnn_get_output_case(sphx_ctx* ctx, int32_t c, double* out) { ENG_CALL(gnn_get_output(c, out)); }

int sphx_gnn_set_target_case(sphx_ctx* ctx, int32_t c, const double* target) { ENG_CALL(gnn_set_target(c, target)); }

int sphx_gnn_train_step(sphx_ctx* ctx, double lr, double* loss) { ENG_CALL(gnn_train_step(lr, loss)); }

int sphx_gnn_profile(sphx_ctx* ctx, int32_t reps, double* ms, int64_t* sizes) { ENG_CALL(gnn_profile(reps, ms, sizes)); }

int sphx_surrogate_advance(sphx_ctx* ctx, int32_t windows, double max_drho, int32_t plain_every, int64_t* n_fallback,
                           int64_t* n_surrogate)
{
    ENG_CALL(surrogate_advance(windows, max_drho, plain_every, n_fallback, n_surrogate));
}

}  // extern "C"
