// sphx_device.hpp -- HIP kernels (gfx950) of the Riemann-based weakly
// compressible SPH step of the SPHinXsys paper (arXiv 2010.12375):
// cell binning and neighbour configuration (Section 9, cell-linked list and
// neighbour relation), density re-initialisation (Eq. eqrhosum), Riemann
// pressure and density relaxation with one-sided wall states (Eqs.
// riemannsph, eqriepartial, eqrienoslip, eqriepright), dual-criteria time
// steps (Eqs. dt-advection, dt-relax) and position-based Verlet (Section 7).
//
// One launch serves a batch of independent cases, each a fluid body and a
// wall body (static, or moving with a prescribed rigid motion) with its own
// parameters, clock and time steps. Every case
// owns whole tiles of TILE consecutive particle slots, so a wavefront (and a
// block of a pair kernel) never spans two cases: the case and its parameters
// are uniform and come from the parameter table with scalar loads.
//
// Data layout (cases concatenated; inside a case cell-sorted particle order;
// structure of arrays for what a thread reads only for itself, small packed
// records for what neighbours gather):
//   x[k]   double   position accumulators, one array per axis
//   geo    R2/R4    FP32 (or FP64) offset of the configuration-time position
//                   from the origin of its cell: the frozen pair geometry is
//                   recomputed from these as (o_i - o_j) - dc L, which keeps
//                   FP32 relative error near 1e-7 of a cell instead of 1e-7
//                   of the domain
//   st     R4       {v0, v1, dev, drho} in 2D, {v0, v1, v2, dev} in 3D, with
//                   dev = rho - rho0 (the density deviation carries the
//                   pressure p = c^2 dev without the cancellation of rho - rho0)
//   dr3    real     drho/dt in 3D
//   hf     R4       {vn.., dev_half}: v^{n+1} and rho^{n+1/2} - rho0 written by
//                   the pressure relaxation for the density relaxation
//   nbr    u32      neighbour entries, wave-tiled (ell_at): sorted index |
//                   stencil code << 26, the code holding the cell offset
//                   dc + 1 (2 bits per axis)
// Cells: case c owns global cells [cbase, cbase + ncell) and one padding cell
// cbase + ncell that holds its unused slots, so one counting sort over all
// cells leaves every case on its own slot range.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sphx {

constexpr int NBR_SHIFT = 26;
constexpr uint32_t NBR_MASK = (1u << NBR_SHIFT) - 1u;
constexpr int TILE = 64;    // particle slots per tile; cases own whole tiles
constexpr int BLOCK = 256;  // threads per block of every particle kernel
#ifndef SPHX_PAIR_BATCH
#define SPHX_PAIR_BATCH 4
#endif
constexpr int BATCH = SPHX_PAIR_BATCH;  // list entries loaded ahead per lane (pair kernels)
#ifndef SPHX_BUILD_BATCH
#define SPHX_BUILD_BATCH 4
#endif
constexpr int NBATCH = SPHX_BUILD_BATCH;  // candidate rounds loaded ahead per lane (neighbour build)
// Inside a cell the particles are ordered by x sub-bin (XSUB bins of width
// L/XSUB along x), then by previous slot. The sub-bin rides in the bits above
// CELL_BITS of a slot's cell word and binning key (global cell indices stay
// below 2^CELL_BITS); per cell, the cumulative sub-bin counts let the
// neighbour build skip the parts of the outer cells of a stencil row that lie
// beyond 2h in x.
constexpr int XSUB = 4;
constexpr int CELL_BITS = 28;
constexpr int32_t CELL_MASK = (1 << CELL_BITS) - 1;
constexpr int VSLOTS = 64;  // slots the density relaxation folds its block maxima into
#ifndef SPHX_PAIR_WAVES
#define SPHX_PAIR_WAVES 0
#endif
#ifndef SPHX_PREFETCH_3D
#define SPHX_PREFETCH_3D 0
#endif
#if SPHX_PAIR_WAVES > 0
#define SPHX_PAIR_ATTR __attribute__((amdgpu_waves_per_eu(SPHX_PAIR_WAVES)))
#else
#define SPHX_PAIR_ATTR
#endif

enum : uint32_t {
    ERR_ESCAPE = 1u,       // a fluid particle left the domain box
    ERR_NAN = 2u,          // NaN in the state
    ERR_NBR_OVERFLOW = 4u, // neighbour list capacity exceeded
};

// State of one acoustic sub-step; sub-step q of a queue lives in
// Ctrl::ss[q & 1]. The pressure relaxation of sub-step q derives it from
// sub-step q - 1 (every block of the case computes the same values, the
// case's first block stores them), so no kernel reads a slot that the same
// launch writes.
struct SubState {
    double tau;      // time covered inside the advection step before this sub-step
    double dt;       // size of this sub-step
    int32_t last;    // this sub-step ends the advection step
    int32_t active;  // this sub-step is to be done
    int32_t nsub;    // sub-steps done in the advection step before this one
    int32_t pad;
};

// Device-side control block of one case's time loop.
struct Ctrl {
    double t;          // clock (time of the current state)
    double t_end;      // end of the current advection step
    double t_stop;     // caller's stop time
    double dt_ad;      // current advection step size
    double vmax;       // |v|max of the current state
    unsigned long long vmax_bits;  // scratch of k_vmax
    SubState ss[2];
    int32_t midstep;   // the advection step continues in the next queue (its state is in ss[0])
    int32_t rebuild;   // an advection step ended in this queue: update the configuration
    long long nsub_total;
    long long steps_done;
    long long steps_target;  // no advection step starts once steps_done reaches it
    uint32_t err;         // sticky error bits; no kernel that tests them also sets them
    uint32_t err_pending; // bits raised by the density relaxation, folded into err later
};

template <typename real> struct alignas(4 * sizeof(real)) R4 { real x, y, z, w; };
template <typename real> struct alignas(2 * sizeof(real)) R2 { real x, y; };
template <typename real> __device__ __forceinline__ real zc(const R2<real>&) { return (real)0; }
template <typename real> __device__ __forceinline__ real zc(const R4<real>& v) { return v.z; }
template <typename real> __device__ __forceinline__ real geo_w(const R2<real>&) { return (real)0; }
template <typename real> __device__ __forceinline__ real geo_w(const R4<real>& v) { return v.w; }
template <int D, typename real> struct GeoSel { using T = R2<real>; };
template <typename real> struct GeoSel<3, real> { using T = R4<real>; };

// Parameters of one case (device table, one entry per case).
template <typename real> struct KP {
    real rho0, c, c2, inv_c2, half_inv_c;     // EoS and Riemann
    real two_m, m, two_vw, vw;                // particle mass and wall volume
    double md;                                // particle mass in FP64 (diagnostics)
    real inv_h, Wc, dWc;                      // Wendland: Wc = a/h^d, dWc = -5a/h^(d+1)
    real s_r, dWr;                            // -1/(2h), dWc/h: dW/dr = dWr r (1 + s_r r)^3
    real quarter_c;                           // c/4 (bound of the limiter beta/4)
    real g[3];
    real L[3];                                // cell size per axis
    double Ld[3], lo[3], hi[3], period[3], half_period[3];
    int n[3], periodic[3];
    int band;                                 // rows of cells per band of the cell order (see cell_index)
    double rc2, sigma0, rho0d;
    double cfl_ad_h, cfl_ac_h, u_ref, c0d;
    int maxn, maxw;                           // list capacity per particle (same for every case)
    int xsub_margin;                          // 0 if L_x > 2h (beyond rounding), else 1 sub-bin of slack
    real eta, p0;                             // dynamic viscosity, transport background pressure
    double visc_dt;                           // CFL_ad h^2 / nu (0: inviscid)
    int reinit_mode;                          // 0: free surface (max), 1: no free surface
    int adv_forces;                           // eta > 0 or p0 != 0
    int wmove;                                // the walls follow the prescribed motion below
    int wvel;                                 // the walls carry given velocities (surface sliding)
    double wamp[3], womega, wroll, wpivot[3]; // sway amp sin(w t), roll sin(w t) about pivot + sway
    int case_id;
    int fbase, nf, fcap;                      // fluid slots [fbase, fbase + fcap), the first nf used
    int wbase, nw;                            // wall slots [wbase, wbase + nw)
    int cbase, ncell;                         // cells [cbase, cbase + ncell), padding cell cbase + ncell
};

// Neighbour lists are wave-tiled: the 64/T particles served by one
// wavefront (T lanes each) store their entries so that every round of the
// pair loop reads 64 consecutive words: entry k of particle i sits at word
// (k mod T) + T (i mod 64/T) + 64 (k div T) of the tile of particle i, tiles
// holding mx entries per particle.
template <int T>
__host__ __device__ __forceinline__ size_t ell_at(int i, int k, int mx)
{
    constexpr int PW = 64 / T;
    size_t tile = (size_t)(i / PW);
    int p = i % PW;
    return (tile * (size_t)(mx / T) + (size_t)(k / T)) * 64 + (size_t)p * T + (size_t)(k % T);
}

// The same address split into a per-particle base and a per-entry offset
// (unsigned shifts for the power-of-two T), for loops that write many
// entries of one particle.
template <int T>
__device__ __forceinline__ size_t ell_base(int i, int mx)
{
    constexpr unsigned PW = 64 / T;
    const unsigned ui = (unsigned)i;
    return ((size_t)(ui / PW) * (size_t)((unsigned)mx / T)) * 64 + (size_t)((ui % PW) * T);
}
template <int T>
__device__ __forceinline__ unsigned ell_off(unsigned k)
{
    return (k / T) * 64u + (k % T);
}

// XCD-aware block order. Workgroups are dispatched round-robin over the 8
// XCDs, each with its own L2; remapping so that XCD k runs the k-th
// contiguous slice of the (cell-sorted) particle range keeps neighbouring
// particles, which gather the same neighbour data, on one L2. A bijection on
// [0, nb) for any nb.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_block(int b, int nb)
{
    const int x = b % NXCD, k = b / NXCD;
    const int q = nb / NXCD, rem = nb % NXCD;
    return k + x * q + (x < rem ? x : rem);
}

// Tile of the calling wavefront in a one-thread-per-slot launch of BLOCK
// threads (uniform over the wavefront).
__device__ __forceinline__ int wave_tile()
{
    return __builtin_amdgcn_readfirstlane((int)((blockIdx.x * (unsigned)BLOCK + threadIdx.x) >> 6));
}

// ---------------------------------------------------------------------
// small helpers

template <typename T> __device__ __forceinline__ T dmax(T a, T b) { return a > b ? a : b; }
template <typename T> __device__ __forceinline__ T dmin(T a, T b) { return a < b ? a : b; }
// x clamped to [0, hi] for hi >= 0 (FP32: one median-of-three instruction)
__device__ __forceinline__ float clamp0(float x, float hi) { return __builtin_amdgcn_fmed3f(x, 0.0f, hi); }
__device__ __forceinline__ double clamp0(double x, double hi) { return dmin(dmax(x, 0.0), hi); }

// hardware reciprocal square root (about 1 ulp), far inside the FP32 budget
__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }
// Quotients inside the pair loops: in FP32 a times the hardware reciprocal
// of b (within about 1 ulp of the reciprocal; two instructions instead of
// the correctly rounded division's eleven), in FP64 the division itself.
__device__ __forceinline__ float div_r(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double div_r(double a, double b) { return a / b; }

__device__ __forceinline__ unsigned long long speed_bits(float s) { return (unsigned long long)__float_as_uint(s); }
__device__ __forceinline__ unsigned long long speed_bits(double s) { return (unsigned long long)__double_as_longlong(s); }
template <typename real> __device__ __forceinline__ double bits_speed(unsigned long long b);
template <> __device__ __forceinline__ double bits_speed<float>(unsigned long long b) { return (double)__uint_as_float((uint32_t)b); }
template <> __device__ __forceinline__ double bits_speed<double>(unsigned long long b) { return __longlong_as_double((long long)b); }

__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Sum over the T lanes of a group (groups are aligned inside the wavefront).
template <int T>
__device__ __forceinline__ float group_sum(float v)
{
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
template <int T>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int o = T / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Cell coordinate along axis k, clamped into the case's grid (NaN and
// infinities included, so a bad position still yields a valid cell).
template <typename real>
__device__ __forceinline__ int cell_coord(const KP<real>& P, int k, double xk)
{
    double f = floor((xk - P.lo[k]) / P.Ld[k]);
    if (!(f >= 0.0)) f = 0.0;
    if (f > (double)(P.n[k] - 1)) f = (double)(P.n[k] - 1);
    return (int)f;
}

// x sub-bin of a position in x cell cx: floor(XSUB t) - XSUB cx with
// t = (x - lo) / L (the quotient cell_coord floors; scaling by the power of
// two XSUB is exact), clamped to [0, XSUB) for the clamped edge cells.
template <typename real>
__device__ __forceinline__ int xsub_bin(const KP<real>& P, double x, int cx)
{
    const double f = floor((x - P.lo[0]) / P.Ld[0] * (double)XSUB) - (double)XSUB * (double)cx;
    return f < 0.0 ? 0 : (f > (double)(XSUB - 1) ? XSUB - 1 : (int)f);
}

// Particles of a cell below / above an x sub-bin, from the cell's packed
// cumulative counts w (byte b: particles with sub-bin <= b for b < XSUB - 1,
// top byte: all; 0 where the cell is empty or holds more than 255).
__device__ __forceinline__ int xsub_below(uint32_t w, int b)
{
    return b <= 0 ? 0 : (int)((w >> (8 * (b - 1))) & 0xffu);
}
__device__ __forceinline__ int xsub_above(uint32_t w, int b)
{
    return b >= XSUB - 1 ? 0 : (int)(w >> 24) - (int)((w >> (8 * b)) & 0xffu);
}

// Cell order. Each row of cells along x is contiguous (the neighbour build
// scans three x-adjacent cells as one range). Rows are grouped into bands of
// `band` rows along y and ordered band by band, inside a band by z, then y.
// With a single z layer (2D) this is plain row-major order. In 3D it keeps
// the rows a particle's neighbours lie in (y +- 1, z +- 1) within about
// band * n_x cells of its own row, except at band edges, instead of a whole
// x-y layer away, so that the neighbour records the wavefronts of one XCD
// gather stay in that XCD's L2.
template <typename real>
__device__ __forceinline__ int cell_row(const KP<real>& P, int c1, int c2)
{
    const int b = c1 / P.band;
    const int rows = min(P.band, P.n[1] - b * P.band);
    return b * P.band * P.n[2] + c2 * rows + (c1 - b * P.band);
}

template <typename real>
__device__ __forceinline__ int cell_index(const KP<real>& P, int c0, int c1, int c2)
{
    return P.n[0] * cell_row(P, c1, c2) + c0;
}

// Inverse of cell_index for a cell of the case (local index lc).
template <typename real>
__device__ __forceinline__ void cell_coords(const KP<real>& P, int lc, int c[3])
{
    const int row = lc / P.n[0];
    c[0] = lc - row * P.n[0];
    const int full = P.n[1] / P.band, per = P.band * P.n[2];
    int b = row / per, rows = P.band, rem = row - b * per;
    if (b >= full) {  // the last, partial band
        b = full;
        rows = P.n[1] - full * P.band;
        rem = row - full * per;
    }
    c[2] = rem / rows;
    c[1] = b * P.band + (rem - c[2] * rows);
}

// FP64 neighbour predicate on absolute positions: dx = x_i - x_j with one
// minimum-image wrap on periodic axes, r^2 summed left to right, no FMA.
template <int D, typename real>
__device__ __forceinline__ double pair_r2(const KP<real>& P, const double* xi, const double* xj)
{
#pragma clang fp contract(off)
    double t[3];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double u = xi[k] - xj[k];
        if (P.periodic[k]) {
            if (u > P.half_period[k]) u -= P.period[k];
            else if (u < -P.half_period[k]) u += P.period[k];
        }
        t[k] = u;
    }
    double r2 = t[0] * t[0] + t[1] * t[1];
    if (D == 3) r2 = r2 + t[2] * t[2];
    return r2;
}

// Frozen pair geometry from cell offsets: d = x_i - x_j, 1/r_ij, r_ij,
// e_ij = -d/r (from i to j) and dW/dr of the Wendland C2 kernel with
// support 2h. The pair loops use d and 1/r where that saves the products of
// e (e.g. (v_i - v_j) . e_ij = -(v_i - v_j) . d / r); the compiler drops
// what a caller does not use. A neighbour's cell code c in {0, 1, 2} per
// axis enters as d = (o_i - o_j) - (c - 1) L.
template <int D, typename real> struct Pair {
    real d[3];
    real rinv;
    real e[3];
    real r;
    real dW;
    real dW_r;  // dW/dr / r
};

// The same from the cell offset vector c = (dc_x L_x, dc_y L_y, dc_z L_z)
// of the entry's stencil code, read from a per-block table (CellOffsets):
// (o_i - o_j) - c equals (o_i - o_j) - dc L bit for bit (dc L is exact), and
// saves the code's decoding per pair.
template <int D, typename real, typename G>
__device__ __forceinline__ Pair<D, real> pair_geo_c(const KP<real>& P, const G& oi, const G& oj, const R4<real>& c)
{
    Pair<D, real> q;
    real* dx = q.d;
    dx[0] = (oi.x - oj.x) - c.x;
    dx[1] = (oi.y - oj.y) - c.y;
    if constexpr (D == 3) dx[2] = (oi.z - zc(oj)) - c.z;
    else dx[2] = (real)0;
    real r2 = dx[0] * dx[0] + dx[1] * dx[1] + (D == 3 ? dx[2] * dx[2] : (real)0);
    real rinv = rsqrt_r(r2);
    real r = r2 * rinv;
    real s = (real)1 + P.s_r * r;
    q.dW_r = P.dWr * s * s * s;
    q.dW = q.dW_r * r;
    q.r = r;
    q.rinv = rinv;
    q.e[0] = -dx[0] * rinv;
    q.e[1] = -dx[1] * rinv;
    q.e[2] = -dx[2] * rinv;
    return q;
}

// Cell offset vectors of the 64 stencil codes (27 used) for the block's
// case, in LDS: entry c = ((c & 3) - 1) L_x, ((c >> 2 & 3) - 1) L_y,
// ((c >> 4 & 3) - 1) L_z. Filled by the block's first 64 threads; the caller
// synchronises the block before use.
template <typename real>
__device__ __forceinline__ void fill_cell_offsets(const KP<real>& P, R4<real>* tab)
{
    const int c = threadIdx.x;
    if (c < 64) {
        R4<real> v;
        v.x = (real)((c & 3) - 1) * P.L[0];
        v.y = (real)(((c >> 2) & 3) - 1) * P.L[1];
        v.z = (real)(((c >> 4) & 3) - 1) * P.L[2];
        v.w = (real)0;
        tab[c] = v;
    }
}

template <int D, typename real, typename G>
__device__ __forceinline__ Pair<D, real> pair_geo(const KP<real>& P, const G& oi, const G& oj, uint32_t code)
{
    Pair<D, real> q;
    real* dx = q.d;
    dx[0] = (oi.x - oj.x) - (real)((int)(code & 3u) - 1) * P.L[0];
    dx[1] = (oi.y - oj.y) - (real)((int)((code >> 2) & 3u) - 1) * P.L[1];
    if constexpr (D == 3) dx[2] = (oi.z - oj.z) - (real)((int)((code >> 4) & 3u) - 1) * P.L[2];
    else dx[2] = (real)0;
    real r2 = dx[0] * dx[0] + dx[1] * dx[1] + (D == 3 ? dx[2] * dx[2] : (real)0);
    real rinv = rsqrt_r(r2);
    real r = r2 * rinv;
    // listed pairs have r < 2h (up to the rounding of r), so 1 - r/(2h) >= 0
    real s = (real)1 + P.s_r * r;
    q.dW_r = P.dWr * s * s * s;
    q.dW = q.dW_r * r;
    q.r = r;
    q.rinv = rinv;
    q.e[0] = -dx[0] * rinv;
    q.e[1] = -dx[1] * rinv;
    q.e[2] = -dx[2] * rinv;
    return q;
}

// Moving walls (Section 2.3 with u_w != 0). A case's wall body follows a
// prescribed rigid motion: displacement d(t) = amp sin(w t) and rotation
// theta(t) = roll sin(w t) in the x-y plane about the moving centre
// pivot + d(t). Wall particles with flag 0 stay where they were given.
// The pose is taken at each configuration update and frozen with the rest
// of the configuration; the velocity rates d'(t), theta'(t) are evaluated
// at each relaxation's time level. The pose is computed without FP
// contraction in the operation order the definition is written in.
template <typename real>
__device__ __forceinline__ void wall_pose(const KP<real>& P, double t, int moving, const double x0[3],
                                          const double n0[3], double x[3], double n[3])
{
#pragma clang fp contract(off)
    if (!P.wmove || !moving) {
        for (int k = 0; k < 3; ++k) {
            x[k] = x0[k];
            n[k] = n0[k];
        }
        return;
    }
    const double sn = sin(P.womega * t);
    const double th = P.wroll * sn;
    const double ct = cos(th), st = sin(th);
    const double d0 = x0[0] - P.wpivot[0], d1 = x0[1] - P.wpivot[1];
    x[0] = (P.wpivot[0] + P.wamp[0] * sn) + (ct * d0 - st * d1);
    x[1] = (P.wpivot[1] + P.wamp[1] * sn) + (st * d0 + ct * d1);
    x[2] = (P.wpivot[2] + P.wamp[2] * sn) + (x0[2] - P.wpivot[2]);
    n[0] = ct * n0[0] - st * n0[1];
    n[1] = st * n0[0] + ct * n0[1];
    n[2] = n0[2];
}

// Translation velocity d'(t) and rotation rate theta'(t) of the wall motion.
template <typename real>
__device__ __forceinline__ void wall_rates(const KP<real>& P, double t, real V[3], real& om)
{
    const double co = cos(P.womega * t);
    V[0] = (real)(P.wamp[0] * P.womega * co);
    V[1] = (real)(P.wamp[1] * P.womega * co);
    V[2] = (real)(P.wamp[2] * P.womega * co);
    om = (real)(P.wroll * P.womega * co);
}

// Velocity of a wall particle from its motion record k = {m r_x, m r_y, m, 0}
// (m: follows the motion, r: lever arm from the rotation centre at the
// configuration update): v_w = m d'(t) + theta'(t) z x (m r).
template <typename real>
__device__ __forceinline__ void wall_velocity(const R4<real>& k, const real V[3], real om, real v[3])
{
    v[0] = k.z * V[0] - om * k.y;
    v[1] = k.z * V[1] + om * k.x;
    v[2] = k.z * V[2];
}

// Add a wall particle's given velocity g = {v_x, v_y, v_z, 0}.
template <typename real>
__device__ __forceinline__ void add_given(const R4<real>& g, real v[3])
{
    v[0] += g.x;
    v[1] += g.y;
    v[2] += g.z;
}

// Whether the case of the tile holding slot i0 has walls with a velocity
// (a motion or given velocities).
template <typename real>
__device__ __forceinline__ bool wall_velocity_case(const KP<real>* __restrict__ Pt,
                                                   const int32_t* __restrict__ tcase, int i0)
{
    const KP<real>& P = Pt[tcase[i0 / TILE]];
    return P.wmove || P.wvel;
}

// Density re-initialisation of one particle from its kernel sum sigma (self
// included): rho = max(rho*, rho0 sigma / sigma0) for free-surface flow,
// rho0 sigma / sigma0 without free surface; st holds rho - rho0.
template <int D, typename real>
__device__ __forceinline__ void reinit_density(const KP<real>& P, double sigma, R4<real>* __restrict__ sp)
{
    const real dev_sum = (real)(P.rho0d * (sigma / P.sigma0 - 1.0));
    R4<real> s = *sp;
    if (D == 2) {
        if (P.reinit_mode || dev_sum > s.z) { s.z = dev_sum; *sp = s; }
    } else {
        if (P.reinit_mode || dev_sum > s.w) { s.w = dev_sum; *sp = s; }
    }
}

template <typename real>
__device__ __forceinline__ real kernel_W(const KP<real>& P, real r)
{
    real qh = r * P.inv_h;
    real s = dmax((real)1 - (real)0.5 * qh, (real)0);
    return P.Wc * s * s * s * s * ((real)1 + (real)2 * qh);
}

// A case updates its configuration when one of its advection steps ended in
// the queue just run (or on request, `force`); otherwise its cells, order,
// frozen geometry and lists are kept, and the sort below is the identity on
// its slots. The decision is read from state no kernel of the update writes.
__device__ __forceinline__ bool full_update(const Ctrl* ctrl, int force) { return force || ctrl->rebuild; }

// ---------------------------------------------------------------------
// S1: cell binning (one stable counting sort over the cells of all cases)

// Wrap periodic coordinates, check escapes, compute the global cell key and
// an arrival rank inside the cell (one thread per slot). The last tile of a
// case puts the case's unused slots into its padding cell. At the end of a
// queue (q >= 0) each wavefront decides itself whether its case takes a full
// update (update_due); escape and NaN bits go to err_pending, which the
// scan's step_end folds in.
template <typename real> __device__ __forceinline__ bool update_due(const KP<real>&, const Ctrl* __restrict__, int,
                                                                    int);

// Bin the slots [i0, i0 + n) of one case (n <= 64), one per lane of the
// calling wavefront: full update from the positions, else the kept cell.
template <int D, typename real>
__device__ __forceinline__ void bin_slots(const KP<real>& P, Ctrl* __restrict__ ctrl, bool full, int i0, int n,
                                          double* __restrict__ x0, double* __restrict__ x1, double* __restrict__ x2,
                                          const int32_t* __restrict__ cell, int32_t* __restrict__ key,
                                          int32_t* __restrict__ rank, int32_t* __restrict__ cnt)
{
    const int lane = threadIdx.x & 63;
    const int i = i0 + lane;
    if (lane == 0 && i0 % TILE == 0 && i0 + TILE == P.fbase + P.fcap) cnt[P.cbase + P.ncell] = P.fcap - P.nf;
    const bool act = lane < n && i < P.fbase + P.nf;  // the active lanes are a prefix of the wavefront
    int kc = -1, sb = 0;
    if (!act) {
    } else if (!full) {
        kc = cell[i] & CELL_MASK;
        sb = (int)((uint32_t)cell[i] >> CELL_BITS);
    } else {
        double* xs[3] = {x0, x1, x2};
        int c[3] = {0, 0, 0};
        uint32_t bad = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double xk = xs[k][i];
            if (xk != xk) bad |= ERR_NAN;
            if (P.periodic[k]) {
                double w = xk;
                if (w >= P.hi[k]) w -= P.period[k];
                else if (w < P.lo[k]) w += P.period[k];
                if (w != xk) { xs[k][i] = w; xk = w; }
            }
            if (!(xk >= P.lo[k] && xk < P.hi[k])) bad |= ERR_ESCAPE;
            c[k] = cell_coord(P, k, xk);
            if (k == 0) sb = xsub_bin(P, xk, c[0]);
        }
        if (bad) atomicOr(&ctrl->err_pending, bad);
        kc = P.cbase + cell_index(P, c[0], c[1], c[2]);
    }
    // Arrival ranks, one atomic per run of equal keys among consecutive
    // lanes (the slots are in the previous cell order, so runs are long):
    // the run's head adds the run length, each lane takes head's base plus
    // its distance from the head. Any dense ranking serves; the placement
    // restores the stable order.
    const int prev = __shfl_up(kc, 1);
    const bool head = act && (lane == 0 || prev != kc);
    const unsigned long long heads = __ballot(head);
    const int nact = __popcll(__ballot(act));
    const unsigned long long le = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const int h = act ? 63 - __clzll(heads & le) : lane;
    int base = 0;
    if (head) {
        const unsigned long long after = heads & ~le;
        const int next = after ? __ffsll((long long)after) - 1 : nact;
        base = atomicAdd(&cnt[kc], next - lane);
    }
    base = __shfl(base, h);
    if (!act) return;
    key[i] = kc | (sb << CELL_BITS);
    rank[i] = base + (lane - h);
}

template <int D, typename real>
__global__ __launch_bounds__(BLOCK) void k_bin(const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase,
                                               int ntiles, Ctrl* __restrict__ ctrl_all, int force,
                                               double* __restrict__ x0, double* __restrict__ x1,
                                               double* __restrict__ x2, const int32_t* __restrict__ cell,
                                               int32_t* __restrict__ key, int32_t* __restrict__ rank,
                                               int32_t* __restrict__ cnt, int q)
{
    const int tile = wave_tile();
    if (tile >= ntiles) return;
    const KP<real>& P = Pt[tcase[tile]];
    Ctrl* ctrl = ctrl_all + P.case_id;
    bin_slots<D>(P, ctrl, update_due(P, ctrl, force, q), tile * TILE, TILE, x0, x1, x2, cell, key, rank, cnt);
}

// Exclusive scan of cell counts in three passes (block sums, scan of block
// sums, add); SCAN_ITEMS consecutive cells per thread.
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = BLOCK * SCAN_ITEMS;

__device__ __forceinline__ int block_excl_scan(int v, int* sh, int& total)
{
    // Hillis-Steele over the block in LDS (BLOCK = 256)
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int o = 1; o < BLOCK; o <<= 1) {
        int a = t >= o ? sh[t - o] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    total = sh[BLOCK - 1];
    int incl = sh[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(BLOCK) void k_scan_tiles(int32_t* __restrict__ cnt, int32_t* __restrict__ start,
                                                      int32_t* __restrict__ bsum, int n)
{
    __shared__ int sh[BLOCK];
    int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        v[q] = base + q < n ? cnt[base + q] : 0;
        s += v[q];
    }
    // the counts are consumed here: leave them zeroed for the next binning
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q)
        if (base + q < n) cnt[base + q] = 0;
    int total;
    int ex = block_excl_scan(s, sh, total);
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q) {
        if (base + q < n) start[base + q] = ex;
        ex += v[q];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

__global__ __launch_bounds__(BLOCK) void k_scan_top(int32_t* __restrict__ bsum, int nb)
{
    __shared__ int sh[BLOCK];
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += BLOCK) {
        int i = b0 + threadIdx.x;
        int v = i < nb ? bsum[i] : 0;
        int total;
        int ex = block_excl_scan(v, sh, total);
        if (i < nb) bsum[i] = ex + carry;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(BLOCK) void k_scan_add(int32_t* __restrict__ start, const int32_t* __restrict__ bsum,
                                                    int n, int nb)
{
    int base = blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int off = bsum[blockIdx.x];
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; ++q)
        if (base + q < n) start[base + q] += off;
    if (blockIdx.x == 0 && threadIdx.x == 0) start[n] = bsum[nb];
}

// Arrival-order list of each cell's fluid particles: slot | sub-bin <<
// CELL_BITS (slots stay below 2^CELL_BITS).
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_scatter(const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase,
                                                   int ntiles, int n, const int32_t* __restrict__ key,
                                                   const int32_t* __restrict__ rank,
                                                   const int32_t* __restrict__ start, int32_t* __restrict__ perm)
{
    const int tile = wave_tile();
    if (tile >= ntiles) return;
    const KP<real>& P = Pt[tcase[tile]];
    const int i = tile * TILE + (threadIdx.x & 63);
    if (i >= P.fbase + P.nf) return;
    const int kw = key[i];
    int p = start[kw & CELL_MASK] + rank[i];
    if (p < n) perm[p] = i | (kw & ~CELL_MASK);  // always true for consistent counts
}

// Stable placement: a particle's slot in its new cell is the number of
// particles of that cell before it in (x sub-bin, previous index) order
// (counted over the cell's arrival-order list from k_scatter), the order of a
// stable counting sort by (cell, sub-bin). The particle that lands first in
// its cell stores the cell's cumulative sub-bin counts. The particle's state
// moves there; with a full update the configuration geometry is frozen anew
// as offsets from the cell origin, otherwise (identity placement: the kept
// cells and sub-bins are already in this order) the frozen offsets move
// along.
template <int D, typename real>
__global__ __launch_bounds__(BLOCK) void k_place_fluid(
    const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase, int ntiles,
    const Ctrl* __restrict__ ctrl_all, int force, int n, const int32_t* __restrict__ arrival,
    const int32_t* __restrict__ key, const int32_t* __restrict__ start, const double* __restrict__ ax0,
    const double* __restrict__ ax1, const double* __restrict__ ax2, const R4<real>* __restrict__ ast,
    const real* __restrict__ adr, const int32_t* __restrict__ aid, const typename GeoSel<D, real>::T* __restrict__ ageo,
    double* __restrict__ bx0, double* __restrict__ bx1, double* __restrict__ bx2, R4<real>* __restrict__ bst,
    real* __restrict__ bdr, int32_t* __restrict__ bid, int32_t* __restrict__ bcell,
    typename GeoSel<D, real>::T* __restrict__ bgeo, uint32_t* __restrict__ xcum)
{
    const int tile = wave_tile();
    if (tile >= ntiles) return;
    const KP<real>& P = Pt[tcase[tile]];
    const bool full = full_update(ctrl_all + P.case_id, force);
    const int i = tile * TILE + (threadIdx.x & 63);
    if (i >= P.fbase + P.nf) return;
    const int kw = key[i];
    const int kc = kw & CELL_MASK;
    const int sb = (int)((uint32_t)kw >> CELL_BITS);
    int s0 = start[kc], s1 = min(start[kc + 1], n);
    int s = s0;
    uint32_t cum = 0;  // byte b: arrivals with sub-bin <= b
    for (int q = s0; q < s1; ++q) {
        const int a = arrival[q];
        const int j = a & CELL_MASK;
        const int sj = (int)((uint32_t)a >> CELL_BITS);
        s += sj < sb || (sj == sb && j < i);
        cum += (0x010101u << (8 * sj)) & 0xffffffu;
    }
    if (s >= n) return;  // never for consistent counts
    if (s == s0) xcum[kc] = s1 - s0 > 255 ? 0u : (cum | ((uint32_t)(s1 - s0) << 24));
    double x[3] = {ax0[i], ax1[i], D == 3 ? ax2[i] : 0.0};
    bx0[s] = x[0];
    bx1[s] = x[1];
    if (D == 3) bx2[s] = x[2];
    bst[s] = ast[i];
    if (D == 3) bdr[s] = adr[i];
    bid[s] = aid[i];
    bcell[s] = kw;
    if (!full) {
        bgeo[s] = ageo[i];
        return;
    }
    int cc[3];
    cell_coords(P, kc - P.cbase, cc);
    const int c0 = cc[0], c1 = cc[1], c2 = cc[2];
    typename GeoSel<D, real>::T g;
    g.x = (real)(x[0] - (P.lo[0] + (double)c0 * P.Ld[0]));
    g.y = (real)(x[1] - (P.lo[1] + (double)c1 * P.Ld[1]));
    if constexpr (D == 3) {
        g.z = (real)(x[2] - (P.lo[2] + (double)c2 * P.Ld[2]));
        g.w = adr[i];  // the density rate rides along (read by the pressure relaxation's gathers)
    }
    bgeo[s] = g;
}

// Walls, sorted by cell at set-up and, for moving walls, at every
// configuration update. Inputs are in the order given (the reference pose);
// `wcase` gives the case of each wall particle, `wflag` whether it follows
// its case's motion. Each wall takes its pose at its case's clock, which
// only changes when the case completes an advection step, so a case that
// does not update its configuration keeps its wall order bit for bit.
template <int D, typename real>
__global__ __launch_bounds__(BLOCK) void k_bin_walls(const KP<real>* __restrict__ Pt, const int32_t* __restrict__ wcase,
                                                     const Ctrl* __restrict__ ctrl_all,
                                                     const int32_t* __restrict__ wflag, int n,
                                                     const double* __restrict__ x0, const double* __restrict__ x1,
                                                     const double* __restrict__ x2, int32_t* __restrict__ key,
                                                     int32_t* __restrict__ rank, int32_t* __restrict__ cnt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const KP<real>& P = Pt[wcase[i]];
    const double xr[3] = {x0[i], x1[i], D == 3 ? x2[i] : 0.0};
    const double nz[3] = {0.0, 0.0, 0.0};
    double xs[3], ns[3];
    wall_pose(P, ctrl_all[P.case_id].t, wflag[i], xr, nz, xs, ns);
    int c[3] = {0, 0, 0};
    for (int k = 0; k < D; ++k) c[k] = cell_coord(P, k, xs[k]);
    int kc = P.cbase + cell_index(P, c[0], c[1], c[2]);
    key[i] = kc;
    rank[i] = atomicAdd(&cnt[kc], 1);
}

__global__ __launch_bounds__(BLOCK) void k_scatter_walls(int n, const int32_t* __restrict__ key,
                                                         const int32_t* __restrict__ rank,
                                                         const int32_t* __restrict__ start, int32_t* __restrict__ perm)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int p = start[key[i]] + rank[i];
    if (p < n) perm[p] = i;
}

// Walls: move into cell order in their pose at the case's clock, freeze
// offsets and normals, keep ids relative to the case's first wall particle.
// One thread per wall particle i (input order): its slot in its cell is the
// number of the cell's wall particles with a smaller input index (counted
// over the cell's arrival list from k_scatter_walls), the order of a stable
// sort, so walls sit in each cell in input order;
// with `bmot`, also the motion record {m r_x, m r_y, m, 0} (m: follows the
// motion, r: lever arm from the rotation centre); with `bvg`, the given
// velocity (vin: 3 per wall particle, input order).
template <int D, typename real>
__global__ __launch_bounds__(BLOCK) void k_gather_wall(
    const KP<real>* __restrict__ Pt, const int32_t* __restrict__ wcase, const Ctrl* __restrict__ ctrl_all,
    const int32_t* __restrict__ wflag, int n, const int32_t* __restrict__ perm, const int32_t* __restrict__ key,
    const int32_t* __restrict__ start, const double* __restrict__ ax0, const double* __restrict__ ax1,
    const double* __restrict__ ax2,
    const double* __restrict__ an0, const double* __restrict__ an1, const double* __restrict__ an2,
    double* __restrict__ bx0, double* __restrict__ bx1, double* __restrict__ bx2,
    typename GeoSel<D, real>::T* __restrict__ bgeo, typename GeoSel<D, real>::T* __restrict__ bnrm,
    int32_t* __restrict__ bid, R4<real>* __restrict__ bmot, const double* __restrict__ vin,
    R4<real>* __restrict__ bvg)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int s0 = start[key[i]], s1 = min(start[key[i] + 1], n);
    int s = s0;
    for (int q = s0; q < s1; ++q) s += perm[q] < i;
    if (s >= n) return;  // never for consistent counts
    const KP<real>& P = Pt[wcase[i]];
    int kc = key[i] - P.cbase;
    const double t = ctrl_all[P.case_id].t;
    const double xr[3] = {ax0[i], ax1[i], D == 3 ? ax2[i] : 0.0};
    const double nr[3] = {an0[i], an1[i], D == 3 ? an2[i] : 0.0};
    double x[3], nv[3];
    const int mv = wflag[i];
    wall_pose(P, t, mv, xr, nr, x, nv);
    if (bmot) {
        R4<real> k = {(real)0, (real)0, (real)0, (real)0};
        if (P.wmove && mv) {
            const double sn = sin(P.womega * t);
            k.x = (real)(x[0] - (P.wpivot[0] + P.wamp[0] * sn));
            k.y = (real)(x[1] - (P.wpivot[1] + P.wamp[1] * sn));
            k.z = (real)1;
        }
        bmot[s] = k;
    }
    if (bvg) bvg[s] = R4<real>{(real)vin[3 * (size_t)i], (real)vin[3 * (size_t)i + 1], (real)vin[3 * (size_t)i + 2],
                               (real)0};
    bx0[s] = x[0];
    bx1[s] = x[1];
    if (D == 3) bx2[s] = x[2];
    bid[s] = i - P.wbase;
    int cc[3];
    cell_coords(P, kc, cc);
    const int c0 = cc[0], c1 = cc[1], c2 = cc[2];
    typename GeoSel<D, real>::T g, nn;
    g.x = (real)(x[0] - (P.lo[0] + (double)c0 * P.Ld[0]));
    g.y = (real)(x[1] - (P.lo[1] + (double)c1 * P.Ld[1]));
    nn.x = (real)nv[0];
    nn.y = (real)nv[1];
    if constexpr (D == 3) {
        g.z = (real)(x[2] - (P.lo[2] + (double)c2 * P.Ld[2]));
        g.w = (real)0;
        nn.z = (real)nv[2];
        nn.w = (real)0;
    }
    bgeo[s] = g;
    bnrm[s] = nn;
}

// Compile-time body selector of the neighbour build (0 fluid, 1 wall).
template <int B> struct BodyTag { static constexpr int value = B; };

// ---------------------------------------------------------------------
// S2: neighbour configuration. For each fluid particle scan the 3^d cells
// around its cell in the fluid and wall cell lists and keep j != i with
// r^2 < (2h)^2, the predicate evaluated exactly as stated on the FP64
// positions. Entries keep the cell offset so that the pair geometry can be
// rebuilt from cell offsets.
//
// TB lanes share one particle; a block is one tile. The three x-adjacent
// cells of a stencil row are one contiguous range of the sorted order; of
// its fluid candidates those in x sub-bins out of reach (below the
// particle's own sub-bin in the left cell, above it in the right one) are
// skipped. The rest is scanned TB candidates per round; hits are appended in
// candidate order
// through a ballot, so the list does not depend on TB. In FP32 mode a
// candidate is first classified on the FP32 cell offsets: |r2_32 - r2| <=
// 6 * 2^-24 L (2 r) + 3 * 2^-24 r^2 < 2.4e-6 L^2 for r <= L (offsets and cell
// sizes rounded once to FP32, then four roundings in the difference), so with
// margin 8e-6 L^2 only candidates in a thin shell around 2h need the FP64
// test, and the list is bit-exact. Cases without a full update keep their
// lists (their order did not change).
//
// With `reinit` (the update at the end of a queue), a case whose next
// advection step has been prepared also gets that step's density
// re-initialisation (Eq. eqrhosum / eqrhosumnosurface) here, saving a
// launch: the kernel sum over the accepted neighbours is taken while they
// are found, from the frozen offsets.
template <int D, typename real, int T, int TB>
__global__ __launch_bounds__(TILE * TB) void k_neighbors(
    const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase, Ctrl* __restrict__ ctrl_all, int force,
    const double* __restrict__ x0, const double* __restrict__ x1, const double* __restrict__ x2,
    const int32_t* __restrict__ cell, const int32_t* __restrict__ fstart,
    const typename GeoSel<D, real>::T* __restrict__ geo, const double* __restrict__ wx0,
    const double* __restrict__ wx1, const double* __restrict__ wx2, const int32_t* __restrict__ wstart,
    const typename GeoSel<D, real>::T* __restrict__ wgeo, uint32_t* __restrict__ nbr, int32_t* __restrict__ ncnt,
    uint32_t* __restrict__ wnb, int32_t* __restrict__ wcnt, int reinit, R4<real>* __restrict__ st,
    const uint32_t* __restrict__ xcum)
{
    static_assert(64 % TB == 0, "lane groups must tile a wavefront");
    using G = typename GeoSel<D, real>::T;
    constexpr bool PREFILTER = sizeof(real) == 4;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const KP<real> P = Pt[tcase[b]];  // a copy: the fields stay in registers through the loops
    Ctrl* ctrl = ctrl_all + P.case_id;
    if (!full_update(ctrl, force) || ctrl->err) return;
    const bool do_reinit = reinit && ctrl->ss[0].active && !ctrl->midstep;
    double sigma = 0.0;
    const int i = b * TILE + (int)threadIdx.x / TB;
    const int l = threadIdx.x % TB;
    const int fend = P.fbase + P.nf, wend = P.wbase + P.nw;
    if (i >= fend) return;  // whole lane groups leave together
    const int gbase = (int)(threadIdx.x & 63) & ~(TB - 1);
    const unsigned long long gmask = TB == 64 ? ~0ull : ((1ull << TB) - 1ull);
    const unsigned long long below = (1ull << l) - 1ull;
    const double xi[3] = {x0[i], x1[i], D == 3 ? x2[i] : 0.0};
    const G oi = geo[i];
    const float Lm = (float)dmax(P.L[0], dmax(P.L[1], D == 3 ? P.L[2] : P.L[1]));
    const float margin = 8e-6f * Lm * Lm;
    const float rc2f = (float)P.rc2;
    const int kc = (cell[i] & CELL_MASK) - P.cbase;
    int ci[3];
    cell_coords(P, kc, ci);
    // fluid candidates of the outer cells of a row lie beyond 2h in x below
    // sub-bin sb_lo of the left cell and above sb_hi of the right one
    const int sb_i = (int)((uint32_t)cell[i] >> CELL_BITS);
    const int sb_lo = sb_i - P.xsub_margin, sb_hi = sb_i + P.xsub_margin;
    int cnt_f = 0, cnt_w = 0;
    uint32_t over = 0;

    // Scan candidates [j0, j1) of one body (fluid: BODY 0, wall: BODY 1, a
    // compile-time constant so that every choice below is static); cell
    // offset in x from the range boundaries b1, b2 (first candidate of the
    // 2nd and 3rd cell).
    auto scan = [&](auto bodyc, int j0, int j1, int b1, int b2, int dcx0, uint32_t tag_yz)
                    __attribute__((always_inline)) {
        constexpr int BODY = decltype(bodyc)::value;
        const G* csrc = BODY ? wgeo : geo;
        const double* bx0 = BODY ? wx0 : x0;
        const double* bx1 = BODY ? wx1 : x1;
        const double* bx2 = BODY ? wx2 : x2;
        const int mx = BODY ? P.maxw : P.maxn;
        uint32_t* out = (BODY ? wnb : nbr) + ell_base<T>(i, mx);
        int& nn = BODY ? cnt_w : cnt_f;
        // NBATCH rounds per iteration: all candidate loads first, then the
        // tests and ballots in candidate order
        for (int jb = j0; jb < j1; jb += TB * NBATCH) {
            G oj[NBATCH];
            double xq[NBATCH][3];
            // unconditional loads (past the end: the range's last candidate,
            // loaded and not tested), so that the NBATCH loads issue back to
            // back without a wait between them
#pragma unroll
            for (int u = 0; u < NBATCH; ++u) {
                const int j = min(jb + u * TB + l, j1 - 1);
                if constexpr (PREFILTER) {
                    oj[u] = csrc[j];
                } else {
                    xq[u][0] = bx0[j];
                    xq[u][1] = bx1[j];
                    xq[u][2] = D == 3 ? bx2[j] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < NBATCH; ++u) {
                if (jb + u * TB >= j1) break;  // uniform over the lane group
                const int j = jb + u * TB + l;
                const int dcx = dcx0 + (j >= b1) + (j >= b2);
                bool in = false;
                float r2w = 0.f;  // FP32 squared distance from the frozen offsets (prefilter)
                if (j < j1 && (BODY || j != i)) {
                    if constexpr (PREFILTER) {
                        float dx = (float)((oi.x - oj[u].x) - (real)dcx * P.L[0]);
                        float dy = (float)((oi.y - oj[u].y) - (real)((int)((tag_yz >> 2) & 3u) - 1) * P.L[1]);
                        float r2 = dx * dx + dy * dy;
                        if constexpr (D == 3) {
                            float dz = (float)((oi.z - zc(oj[u])) - (real)((int)((tag_yz >> 4) & 3u) - 1) * P.L[2]);
                            r2 += dz * dz;
                        }
                        r2w = r2;
                        if (r2 < rc2f - margin) {
                            in = true;
                        } else if (r2 > rc2f + margin) {
                            in = false;
                        } else {
                            double xj[3] = {bx0[j], bx1[j], D == 3 ? bx2[j] : 0.0};
                            in = pair_r2<D>(P, xi, xj) < P.rc2;
                        }
                    } else {
                        in = pair_r2<D>(P, xi, xq[u]) < P.rc2;
                    }
                }
                unsigned long long m = (__ballot(in) >> gbase) & gmask;
                if (in) {
                    int slot = nn + __popcll(m & below);
                    uint32_t code = (uint32_t)(dcx + 1) | tag_yz;
                    if (slot < mx) out[ell_off<T>((unsigned)slot)] = (uint32_t)j | (code << NBR_SHIFT);
                    else over = 1;
                    if (do_reinit) {
                        if constexpr (PREFILTER) {
                            sigma += (double)kernel_W(P, (real)(r2w * rsqrt_r(r2w)));
                        } else {
                            const G ojv = csrc[j];
                            sigma += (double)kernel_W(P, pair_geo<D, real>(P, oi, ojv, code).r);
                        }
                    }
                }
                nn += __popcll(m);
            }
        }
    };

    // One stencil row (three x-adjacent cells) of one body.
    auto row = [&](auto bodyc, int rowc, uint32_t tag_yz) __attribute__((always_inline)) {
        constexpr int BODY = decltype(bodyc)::value;
        const int32_t* st_ = BODY ? wstart : fstart;
        const int lim = BODY ? wend : fend;
        if (ci[0] >= 1 && ci[0] + 1 < P.n[0]) {
            // the three cells are contiguous: one range (fluid: trimmed to
            // the sub-bins within reach)
            const int c = rowc + ci[0];
            int j0 = st_[c - 1], j1 = st_[c + 2];
            if constexpr (BODY == 0) {
                // (the counts of a cell that has emptied are stale: the
                // clamps make them 0)
                j0 = min(j0 + xsub_below(xcum[c - 1], sb_lo), st_[c]);
                j1 = max(j1 - xsub_above(xcum[c + 1], sb_hi), st_[c + 1]);
            }
            scan(bodyc, min(j0, lim), min(j1, lim), min(st_[c], lim), min(st_[c + 1], lim), -1, tag_yz);
        } else {
            for (int dx = -1; dx <= 1; ++dx) {
                int cx = ci[0] + dx;
                if (P.periodic[0]) cx = cx < 0 ? cx + P.n[0] : (cx >= P.n[0] ? cx - P.n[0] : cx);
                else if (cx < 0 || cx >= P.n[0]) continue;
                const int c = rowc + cx;
                scan(bodyc, min(st_[c], lim), min(st_[c + 1], lim), 0x7fffffff, 0x7fffffff, dx, tag_yz);
            }
        }
    };

    const int zlo = D == 3 ? -1 : 0, zhi = D == 3 ? 1 : 0;
    for (int dz = zlo; dz <= zhi; ++dz) {
        int cz = ci[2] + dz;
        if (D == 3) {
            if (P.periodic[2]) cz = cz < 0 ? cz + P.n[2] : (cz >= P.n[2] ? cz - P.n[2] : cz);
            else if (cz < 0 || cz >= P.n[2]) continue;
        }
        for (int dy = -1; dy <= 1; ++dy) {
            int cy = ci[1] + dy;
            if (P.periodic[1]) cy = cy < 0 ? cy + P.n[1] : (cy >= P.n[1] ? cy - P.n[1] : cy);
            else if (cy < 0 || cy >= P.n[1]) continue;
            const int rowc = P.cbase + P.n[0] * cell_row(P, cy, cz);
            const uint32_t tag_yz = ((uint32_t)(dy + 1) << 2) | ((uint32_t)(dz + 1) << 4);
            row(BodyTag<0>{}, rowc, tag_yz);
            if (P.nw > 0) row(BodyTag<1>{}, rowc, tag_yz);
        }
    }
    if (l == 0) {
        ncnt[i] = cnt_f < P.maxn ? cnt_f : P.maxn;
        wcnt[i] = cnt_w < P.maxw ? cnt_w : P.maxw;
    }
    if (over) atomicOr(&ctrl->err, ERR_NBR_OVERFLOW);
    if (do_reinit) {
        sigma = group_sum<TB>(sigma) + (double)P.Wc;  // + W(0), the particle itself
        if (l == 0) reinit_density<D>(P, sigma, st + i);
    }
}

// ---------------------------------------------------------------------
// S5: the dual-criteria clock (Eqs. dt-advection, dt-relax).

// Sub-step 0 of a new advection step (one thread): dt_ad from |v|max floored
// at U_ref and, for viscous flow, the h^2/nu limit, clipped to the stop
// time, and the first acoustic step
// min(dt_ac, dt_ad). Inactive when the clock has reached the stop time, the
// step target is reached or an error is pending.
template <typename real>
__device__ void prepare_step(const KP<real>& P, Ctrl* __restrict__ ctrl)
{
    SubState s0 = {0.0, 0.0, 0, 0, 0, 0};
    const double t = ctrl->t, t_stop = ctrl->t_stop, vmax = ctrl->vmax;
    if (ctrl->err == 0 && t < t_stop && ctrl->steps_done < ctrl->steps_target) {
        double dt_ad = P.cfl_ad_h / fmax(vmax, P.u_ref);
        if (P.visc_dt > 0.0) dt_ad = fmin(dt_ad, P.visc_dt);
        double t_end = t + dt_ad;
        if (t_end >= t_stop) {
            dt_ad = t_stop - t;
            t_end = t_stop;
        }
        double dt_ac = P.cfl_ac_h / (P.c0d + vmax);
        s0.dt = dt_ac;
        if (s0.dt >= dt_ad) {
            s0.dt = dt_ad;
            s0.last = 1;
        }
        s0.active = 1;
        ctrl->dt_ad = dt_ad;
        ctrl->t_end = t_end;
    }
    ctrl->ss[0] = s0;
    ctrl->ss[1].active = 0;
    ctrl->midstep = 0;
}

// The sub-step after S given |v|max of the state S produced: the clock
// advances by S.dt; the next step is min(dt_ac, remaining), the last one
// clipped to land on dt_ad; `finished` when the advection step is covered.
template <typename real>
__device__ __forceinline__ SubState next_substep(const KP<real>& P, double dt_ad, const SubState& S, double vmax,
                                                 bool& finished)
{
    SubState n;
    n.tau = S.tau + S.dt;
    n.nsub = S.nsub + 1;
    n.pad = 0;
    n.dt = S.dt;
    n.last = S.last;
    int done = S.last;
    if (!done) {
        double rem = dt_ad - n.tau;
        if (!(rem > 0.0)) {
            done = 1;
        } else {
            double dt_ac = P.cfl_ac_h / (P.c0d + vmax);
            if (dt_ac >= rem) {
                n.dt = rem;
                n.last = 1;
            } else {
                n.dt = dt_ac;
                n.last = 0;
            }
        }
    }
    n.active = !done;
    finished = done;
    return n;
}

// Bookkeeping of one completed sub-step (one thread).
__device__ __forceinline__ void close_substep(Ctrl* __restrict__ ctrl, int slot, const SubState& n, double vmax,
                                              bool finished)
{
    ctrl->ss[slot] = n;
    ctrl->vmax = vmax;
    ctrl->nsub_total += 1;
    uint32_t pend = ctrl->err_pending;
    if (pend) {
        ctrl->err_pending = 0u;
        ctrl->err |= pend;
    }
    if (finished) {
        ctrl->t = ctrl->t_end;
        ctrl->steps_done += 1;
        ctrl->rebuild = 1;
    }
}

// |v|max of the state a density relaxation produced, from its 64 slots
// (one wavefront; every lane gets the result).
template <typename real>
__device__ __forceinline__ double slot_max(const unsigned long long* __restrict__ vs)
{
    return wave_max(bits_speed<real>(vs[threadIdx.x & 63]));
}

// Start of the advection steps queued by one call (one thread per case); a
// case in the middle of an advection step keeps it.
template <typename real>
__global__ void k_adv_begin(const KP<real>* __restrict__ Pt, Ctrl* __restrict__ ctrl_all, int ncases)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncases) return;
    Ctrl* ctrl = ctrl_all + c;
    if (!ctrl->midstep) prepare_step(Pt[c], ctrl);
}

// Visit the list entries k = l, l + T, ... < n of particle i in batches of
// U: first the U list words (entry l + T r of the lane sits 64 r words past
// its entry l, ell_at, so a batch reads at fixed offsets from one pointer),
// then the U gathers (`load`), then the U updates (`use`), so that several
// memory round trips are in flight per lane. Which entries of a batch exist
// is decided from their index (k < n), so nothing waits on a loaded word to
// know it. Each lane still accumulates its entries in ascending k. The
// lists may be laid out for TL = 2T lanes (the pressure relaxation in 3D
// runs with half the lanes of the layout): entry l + T r then sits in row
// r / 2 at column l + T (r mod 2), still at fixed offsets within a batch.
template <int T, int U, int TL, typename Load, typename Use>
__device__ __forceinline__ void for_pairs(const uint32_t* __restrict__ list, int i, int n, int mx, int l,
                                          Load load, Use use)
{
    static_assert(TL == T || (TL == 2 * T && U % 2 == 0), "layout of T or 2T lanes");
    const uint32_t* q = list + ell_base<TL>(i, mx) + l;
    for (int k0 = l; k0 < n; k0 += T * U, q += 64 * U * T / TL) {
        bool ok[U];
        uint32_t e[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ok[u] = k0 + u * T < n;
            e[u] = 0u;
            if (ok[u]) e[u] = q[TL == T ? 64 * u : 64 * (u >> 1) + T * (u & 1)];
        }
        decltype(load(0u)) g[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (ok[u]) g[u] = load(e[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (ok[u]) use(e[u], g[u]);
    }
}

// Pair kernels: T lanes per particle and pair_threads<T>() threads per
// block (BLOCK, or the T * TILE lanes of one tile where that is fewer), so a
// block lies inside one tile (one case).
template <int T>
__host__ __device__ constexpr int pair_threads()
{
    return T * TILE < BLOCK ? T * TILE : BLOCK;
}

template <int T>
__device__ __forceinline__ int pair_block_first(int b)
{
    static_assert(T >= 1 && T <= 64 && 64 % T == 0, "lane groups must tile a wavefront");
    return b * (pair_threads<T>() / T);
}

// S4: density re-initialisation rho = max(rho*, rho0 sum W / sum W0) with
// the sum over the particle itself, its fluid and its wall neighbours.
// `gate`: only for cases starting an advection step in this queue. T lanes
// share a particle and split its neighbour list.
template <int D, typename real, int T>
__global__ __launch_bounds__(BLOCK) void k_reinit(
    const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase, const Ctrl* __restrict__ ctrl_all, int gate,
    const typename GeoSel<D, real>::T* __restrict__ geo, const typename GeoSel<D, real>::T* __restrict__ wgeo,
    const uint32_t* __restrict__ nbr, const int32_t* __restrict__ ncnt, const uint32_t* __restrict__ wnb,
    const int32_t* __restrict__ wcnt, R4<real>* __restrict__ st)
{
    const int i0 = pair_block_first<T>(xcd_block(blockIdx.x, gridDim.x));
    const KP<real> P = Pt[tcase[i0 / TILE]];  // a copy: the fields stay in registers through the loops
    const Ctrl* ctrl = ctrl_all + P.case_id;
    if (gate && (!ctrl->ss[0].active || ctrl->midstep || ctrl->err)) return;
    const int i = i0 + (int)threadIdx.x / T;
    const int l = threadIdx.x % T;
    if (i >= P.fbase + P.nf) return;
    using G = typename GeoSel<D, real>::T;
    const G oi = geo[i];
    double sigma = 0.0;
    auto add_w = [&](uint32_t e, const G& oj) {
        Pair<D, real> q = pair_geo<D, real>(P, oi, oj, e >> NBR_SHIFT);
        sigma += (double)kernel_W(P, q.r);
    };
    for_pairs<T, BATCH, T>(nbr, i, ncnt[i], P.maxn, l, [&](uint32_t e) { return geo[e & NBR_MASK]; }, add_w);
    for_pairs<T, BATCH, T>(wnb, i, wcnt[i], P.maxw, l, [&](uint32_t e) { return wgeo[e & NBR_MASK]; }, add_w);
    sigma = group_sum<T>(sigma) + (double)P.Wc;  // + W(0), the particle itself
    if (l != 0) return;
    reinit_density<D>(P, sigma, st + i);
}

// Shear force, Eq. (eqviscous), and transport-velocity acceleration,
// Eq. (transport), of each particle on the frozen configuration, once per
// advection step after the re-initialisation (`gate`: for the cases starting
// a step), for the cases that have either:
//   av  = 2 sum_j m eta/(rho_i rho_j) (v_i - v_j)/r W'   (walls: V_w/rho_i, v_j = v_w)
//   atv = 2 sum_j m p0/(rho_i rho_j) W' e_ij             (walls: V_w/rho_i)
// into avt[2 i] and avt[2 i + 1]. T lanes share a particle.
template <int D, typename real, int T, bool MOVE>
__device__ __forceinline__ void adv_forces_body(
    const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase, const Ctrl* __restrict__ ctrl_all, int gate,
    const typename GeoSel<D, real>::T* __restrict__ geo, const typename GeoSel<D, real>::T* __restrict__ wgeo,
    const uint32_t* __restrict__ nbr, const int32_t* __restrict__ ncnt, const uint32_t* __restrict__ wnb,
    const int32_t* __restrict__ wcnt, const R4<real>* __restrict__ st, R4<real>* __restrict__ avt,
    const R4<real>* __restrict__ wmot, const R4<real>* __restrict__ wvg)
{
    const int i0 = pair_block_first<T>(xcd_block(blockIdx.x, gridDim.x));
    const KP<real> P = Pt[tcase[i0 / TILE]];  // a copy: the fields stay in registers through the loops
    const Ctrl* ctrl = ctrl_all + P.case_id;
    if (!P.adv_forces) return;
    if (gate && (!ctrl->ss[0].active || ctrl->midstep || ctrl->err)) return;
    const int i = i0 + (int)threadIdx.x / T;
    const int l = threadIdx.x % T;
    if (i >= P.fbase + P.nf) return;
    using G = typename GeoSel<D, real>::T;
    const G oi = geo[i];
    const R4<real> si = st[i];
    const real vi[3] = {si.x, si.y, D == 3 ? si.z : (real)0};
    const real rho_i = P.rho0 + (D == 2 ? si.z : si.w);
    const real inv_rho_i = (real)1 / rho_i;
    real av[3] = {0, 0, 0}, at[3] = {0, 0, 0};
    // moving walls: velocity at the start of the advection step (no slip),
    // plus the given velocities
    const bool mv = MOVE && P.wmove, gv = MOVE && P.wvel;
    real Vw[3] = {0, 0, 0}, omw = 0;
    if (mv) wall_rates(P, ctrl->t, Vw, omw);
    struct FluidJ { G o; R4<real> s; };
    struct WallJ { G o; R4<real> k, g; };
    for_pairs<T, BATCH, T>(
        nbr, i, ncnt[i], P.maxn, l,
        [&](uint32_t e) {
            uint32_t j = e & NBR_MASK;
            FluidJ r;
            r.o = geo[j];
            r.s = st[j];
            return r;
        },
        [&](uint32_t e, const FluidJ& r) {
            Pair<D, real> q = pair_geo<D, real>(P, oi, r.o, e >> NBR_SHIFT);
            const R4<real>& sj = r.s;
            const real rho_j = P.rho0 + (D == 2 ? sj.z : sj.w);
            const real w = div_r(P.m * inv_rho_i, rho_j) * q.dW;
            const real cv = div_r((real)2 * P.eta * w, q.r);
            const real ct = (real)2 * P.p0 * w;
            av[0] += cv * (vi[0] - sj.x);
            av[1] += cv * (vi[1] - sj.y);
            if (D == 3) av[2] += cv * (vi[2] - sj.z);
            at[0] += ct * q.e[0];
            at[1] += ct * q.e[1];
            if (D == 3) at[2] += ct * q.e[2];
        });
    for_pairs<T, BATCH, T>(
        wnb, i, wcnt[i], P.maxw, l,
        [&](uint32_t e) {
            uint32_t w = e & NBR_MASK;
            WallJ r;
            r.o = wgeo[w];
            if (mv) r.k = wmot[w];
            if (gv) r.g = wvg[w];
            return r;
        },
        [&](uint32_t e, const WallJ& r) {
            Pair<D, real> q = pair_geo<D, real>(P, oi, r.o, e >> NBR_SHIFT);
            const real w = P.vw * inv_rho_i * q.dW;
            const real cv = div_r((real)2 * P.eta * w, q.r);
            const real ct = (real)2 * P.p0 * w;
            real vw[3] = {0, 0, 0};
            if (mv) wall_velocity(r.k, Vw, omw, vw);
            if (gv) add_given(r.g, vw);
            av[0] += cv * (vi[0] - vw[0]);
            av[1] += cv * (vi[1] - vw[1]);
            if (D == 3) av[2] += cv * (vi[2] - vw[2]);
            at[0] += ct * q.e[0];
            at[1] += ct * q.e[1];
            if (D == 3) at[2] += ct * q.e[2];
        });
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        av[k] = group_sum<T>(av[k]);
        at[k] = group_sum<T>(at[k]);
    }
    if (l != 0) return;
    avt[2 * (size_t)i] = R4<real>{av[0], av[1], av[2], (real)0};
    avt[2 * (size_t)i + 1] = R4<real>{at[0], at[1], at[2], (real)0};
}

template <int D, typename real, int T, bool MOVE>
__global__ __launch_bounds__(BLOCK) void k_adv_forces(
    const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase, const Ctrl* __restrict__ ctrl_all, int gate,
    const typename GeoSel<D, real>::T* __restrict__ geo, const typename GeoSel<D, real>::T* __restrict__ wgeo,
    const uint32_t* __restrict__ nbr, const int32_t* __restrict__ ncnt, const uint32_t* __restrict__ wnb,
    const int32_t* __restrict__ wcnt, const R4<real>* __restrict__ st, R4<real>* __restrict__ avt,
    const R4<real>* __restrict__ wmot, const R4<real>* __restrict__ wvg)
{
    if constexpr (MOVE) {
        // cases with static walls run the static instantiation's code
        if (!wall_velocity_case(Pt, tcase, pair_block_first<T>(xcd_block(blockIdx.x, gridDim.x)))) {
            adv_forces_body<D, real, T, false>(
                Pt, tcase, ctrl_all, gate, geo, wgeo, nbr, ncnt, wnb, wcnt, st, avt, wmot, wvg);
            return;
        }
    }
    adv_forces_body<D, real, T, MOVE>(
        Pt, tcase, ctrl_all, gate, geo, wgeo, nbr, ncnt, wnb, wcnt, st, avt, wmot, wvg);
}

// The pair kernels below take MOVE = true only for batches with moving
// walls; the static instantiation compiles none of the wall-velocity code.
// ---------------------------------------------------------------------
// S6: pressure relaxation. First Verlet half-step of density (position
// half-steps are applied together in S7), EoS, Riemann momentum equation
// with fluid and wall neighbours and gravity, velocity update. T lanes share
// a particle: each takes every T-th neighbour, partial sums are combined
// with shuffles and lane 0 writes. TL: the lanes the lists are laid out for
// (T or 2T).
template <int D, typename real, int T, bool MOVE, int TL>
__device__ __forceinline__ void pressure_body(
    const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase, Ctrl* __restrict__ ctrl_all,
    const typename GeoSel<D, real>::T* __restrict__ geo, const typename GeoSel<D, real>::T* __restrict__ wgeo,
    const typename GeoSel<D, real>::T* __restrict__ wnrm, const uint32_t* __restrict__ nbr,
    const int32_t* __restrict__ ncnt, const uint32_t* __restrict__ wnb, const int32_t* __restrict__ wcnt,
    const R4<real>* __restrict__ st, const real* __restrict__ dr3, R4<real>* __restrict__ hf,
    real* __restrict__ acc_out, int q, int adv, unsigned long long* __restrict__ vslot_all,
    const R4<real>* __restrict__ avt, const R4<real>* __restrict__ wmot, const R4<real>* __restrict__ wvg)
{
    const int i0 = pair_block_first<T>(xcd_block(blockIdx.x, gridDim.x));
    const KP<real> P = Pt[tcase[i0 / TILE]];  // a copy: the fields stay in registers through the loops
    Ctrl* ctrl = ctrl_all + P.case_id;
    unsigned long long* vslot = vslot_all + (size_t)P.case_id * 2 * VSLOTS;
    // Sub-step q: with `adv`, first close sub-step q - 1 (every block of the
    // case derives the same state from slot (q - 1) & 1 and the maxima of
    // the last density relaxation; the case's first block stores it in slot
    // q & 1). That block also clears the |v| slots the density relaxation of
    // this sub-step will fill and, at the head of a queue, the update flag.
    // With an error pending no sub-step state is written.
    const uint32_t err = ctrl->err;
    const bool first = i0 == P.fbase;
    SubState S;
    if (adv) {
        const SubState Sp = ctrl->ss[(q - 1) & 1];
        if (Sp.active && !err) {
            const double vmax = slot_max<real>(vslot + ((q - 1) & 1) * VSLOTS);
            bool finished;
            S = next_substep(P, ctrl->dt_ad, Sp, vmax, finished);
            if (first && threadIdx.x == 0) close_substep(ctrl, q & 1, S, vmax, finished);
        } else {
            S = Sp;
            S.active = 0;
            if (first && threadIdx.x == 0 && !err) ctrl->ss[q & 1] = S;
        }
    } else {
        S = ctrl->ss[q & 1];
        if (first && threadIdx.x == 0) ctrl->rebuild = 0;
    }
    if (first && threadIdx.x < VSLOTS) vslot[(q & 1) * VSLOTS + threadIdx.x] = 0ull;
    if (!S.active || err) return;
    __shared__ R4<real> coff[64];
    fill_cell_offsets(P, coff);
    __syncthreads();
    const int i = i0 + (int)threadIdx.x / T;
    const int l = threadIdx.x % T;
    if (i >= P.fbase + P.nf) return;
    using G = typename GeoSel<D, real>::T;
    const real dt = (real)S.dt;
    const real half = (real)0.5 * dt;
    // moving walls: velocity rates at the sub-step's start (the level of v^n),
    // plus the given velocities
    const bool mv = MOVE && P.wmove, gv = MOVE && P.wvel;
    real Vw[3] = {0, 0, 0}, omw = 0;
    if (mv) wall_rates(P, ctrl->t + S.tau, Vw, omw);
    const R4<real> si = st[i];
    real vi[3], dev_i;
    if (D == 2) {
        vi[0] = si.x; vi[1] = si.y; vi[2] = 0;
        dev_i = si.z + half * si.w;
    } else {
        vi[0] = si.x; vi[1] = si.y; vi[2] = si.z;
        dev_i = si.w + half * dr3[i];  // (= geo[i].w)
    }
    const real rho_i = P.rho0 + dev_i;
    const real p_i = P.c2 * dev_i;
    const real inv_rho_i = (real)1 / rho_i;
    const real mi = P.two_m * inv_rho_i;   // 2 m / rho_i
    const real wi = P.two_vw * inv_rho_i;  // 2 V_w / rho_i
    const G oi = geo[i];
    real acc[3] = {0, 0, 0};
    struct FluidJ { G o; R4<real> s; };
    struct WallJ { G o; G n; R4<real> k, g; };
    for_pairs<T, BATCH, TL>(
        nbr, i, ncnt[i], P.maxn, l,
        [&](uint32_t e) {
            uint32_t j = e & NBR_MASK;
            FluidJ r;
            r.o = geo[j];
            r.s = st[j];
            return r;
        },
        [&](uint32_t e, const FluidJ& r) {
            Pair<D, real> pq = pair_geo_c<D, real>(P, oi, r.o, coff[e >> NBR_SHIFT]);
            const R4<real>& sj = r.s;
            // 3D: the neighbour's density rate is the w of its frozen offsets
            real dev_j = D == 2 ? sj.z + half * sj.w : sj.w + half * geo_w(r.o);
            // U_L - U_R = (v_i - v_j) . e_ij = -(v_i - v_j) . d / r
            real dvd = (vi[0] - sj.x) * pq.d[0] + (vi[1] - sj.y) * pq.d[1] +
                       (D == 3 ? (vi[2] - sj.z) * pq.d[2] : (real)0);
            real du = -dvd * pq.rinv;
            real rho_j = P.rho0 + dev_j;
            real p_j = P.c2 * dev_j;
            real qbeta = clamp0((real)0.75 * du, P.quarter_c);  // beta / 4 = min(3 max(du, 0), c) / 4
            real ps = (real)0.5 * (p_i + p_j) + qbeta * (rho_i + rho_j) * du;
            // coef e_ij with coef = 2 m ps W' / (rho_i rho_j), e_ij = -d / r
            real cd = div_r(mi * ps, rho_j) * pq.dW_r;
            acc[0] -= cd * pq.d[0];
            acc[1] -= cd * pq.d[1];
            if (D == 3) acc[2] -= cd * pq.d[2];
        });
    for_pairs<T, BATCH, TL>(
        wnb, i, wcnt[i], P.maxw, l,
        [&](uint32_t e) {
            uint32_t w = e & NBR_MASK;
            WallJ r;
            r.o = wgeo[w];
            r.n = wnrm[w];
            if (mv) r.k = wmot[w];
            if (gv) r.g = wvg[w];
            return r;
        },
        [&](uint32_t e, const WallJ& r) {
            Pair<D, real> pq = pair_geo_c<D, real>(P, oi, r.o, coff[e >> NBR_SHIFT]);
            const G& nw = r.n;
            real UL = -(nw.x * vi[0] + nw.y * vi[1] + (D == 3 ? zc(nw) * vi[2] : (real)0));
            real uw = 0;  // u_w = -n_w . v_w, zero for a static wall
            if (mv || gv) {
                real vw[3] = {0, 0, 0};
                if (mv) wall_velocity(r.k, Vw, omw, vw);
                if (gv) add_given(r.g, vw);
                uw = -(nw.x * vw[0] + nw.y * vw[1] + (D == 3 ? zc(nw) * vw[2] : (real)0));
            }
            real du = (real)2 * (UL - uw);  // U_L - U_R with U_R = -U_L + 2 u_w
            // g . r_fw with r_fw = x_w - x_i = -d
            real gr = -(P.g[0] * pq.d[0] + P.g[1] * pq.d[1] + (D == 3 ? P.g[2] * pq.d[2] : (real)0));
            real pR = p_i + rho_i * gr;
            real rhoR = P.rho0 + pR * P.inv_c2;
            real qbeta = clamp0((real)0.75 * du, P.quarter_c);  // beta / 4
            real ps = (real)0.5 * (p_i + pR) + qbeta * (rho_i + rhoR) * du;
            real cd = wi * ps * pq.dW_r;
            acc[0] -= cd * pq.d[0];
            acc[1] -= cd * pq.d[1];
            if (D == 3) acc[2] -= cd * pq.d[2];
        });
    acc[0] = group_sum<T>(acc[0]);
    acc[1] = group_sum<T>(acc[1]);
    if (D == 3) acc[2] = group_sum<T>(acc[2]);
    if (l != 0) return;
    acc[0] += P.g[0];
    acc[1] += P.g[1];
    acc[2] += P.g[2];
    if (avt && P.adv_forces) {  // shear force of the advection step
        const R4<real> a = avt[2 * (size_t)i];
        acc[0] += a.x;
        acc[1] += a.y;
        acc[2] += a.z;
    }
    R4<real> o;
    o.x = vi[0] + dt * acc[0];
    o.y = vi[1] + dt * acc[1];
    if (D == 2) {
        o.z = dev_i;
        o.w = 0;
    } else {
        o.z = vi[2] + dt * acc[2];
        o.w = dev_i;
    }
    hf[i] = o;
    if (acc_out) {
        acc_out[(size_t)i * D + 0] = acc[0];
        acc_out[(size_t)i * D + 1] = acc[1];
        if (D == 3) acc_out[(size_t)i * D + 2] = acc[2];
    }
}

template <int D, typename real, int T, bool MOVE, int TL = T>
__global__ __launch_bounds__(BLOCK) SPHX_PAIR_ATTR void k_pressure(
    const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase, Ctrl* __restrict__ ctrl_all,
    const typename GeoSel<D, real>::T* __restrict__ geo, const typename GeoSel<D, real>::T* __restrict__ wgeo,
    const typename GeoSel<D, real>::T* __restrict__ wnrm, const uint32_t* __restrict__ nbr,
    const int32_t* __restrict__ ncnt, const uint32_t* __restrict__ wnb, const int32_t* __restrict__ wcnt,
    const R4<real>* __restrict__ st, const real* __restrict__ dr3, R4<real>* __restrict__ hf,
    real* __restrict__ acc_out, int q, int adv, unsigned long long* __restrict__ vslot_all,
    const R4<real>* __restrict__ avt, const R4<real>* __restrict__ wmot, const R4<real>* __restrict__ wvg)
{
    if constexpr (MOVE) {
        // cases with static walls run the static instantiation's code
        if (!wall_velocity_case(Pt, tcase, pair_block_first<T>(xcd_block(blockIdx.x, gridDim.x)))) {
            pressure_body<D, real, T, false, TL>(
                Pt, tcase, ctrl_all, geo, wgeo, wnrm, nbr, ncnt, wnb, wcnt, st, dr3, hf, acc_out, q, adv, vslot_all,
                avt, wmot, wvg);
            return;
        }
    }
    pressure_body<D, real, T, MOVE, TL>(
        Pt, tcase, ctrl_all, geo, wgeo, wnrm, nbr, ncnt, wnb, wcnt, st, dr3, hf, acc_out, q, adv, vslot_all, avt,
        wmot, wvg);
}

// ---------------------------------------------------------------------
// S7: density relaxation. Riemann continuity equation with fluid and wall
// neighbours using v^{n+1}, second Verlet half-steps of position (both
// position half-steps land here, in the paper's order) and density, and the
// block maxima of |v| for the next acoustic step. T lanes share a particle
// as in S6.
template <int D, typename real, int T, bool MOVE>
__device__ __forceinline__ void density_body(
    const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase, Ctrl* __restrict__ ctrl_all, int finalize,
    const typename GeoSel<D, real>::T* __restrict__ geo, const typename GeoSel<D, real>::T* __restrict__ wgeo,
    const typename GeoSel<D, real>::T* __restrict__ wnrm, const uint32_t* __restrict__ nbr,
    const int32_t* __restrict__ ncnt, const uint32_t* __restrict__ wnb, const int32_t* __restrict__ wcnt,
    const R4<real>* __restrict__ hf, R4<real>* __restrict__ st, real* __restrict__ dr3, double* __restrict__ x0,
    double* __restrict__ x1, double* __restrict__ x2, real* __restrict__ drho_out,
    unsigned long long* __restrict__ vslot_all, int q, const R4<real>* __restrict__ avt,
    const R4<real>* __restrict__ wmot, const R4<real>* __restrict__ wvg)
{
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int i0 = pair_block_first<T>(b);
    const KP<real> P = Pt[tcase[i0 / TILE]];  // a copy: the fields stay in registers through the loops
    Ctrl* ctrl = ctrl_all + P.case_id;
    const SubState S = ctrl->ss[q & 1];
    if (!S.active || ctrl->err) return;
    __shared__ double smax[BLOCK / 64];
    __shared__ R4<real> coff[64];
    fill_cell_offsets(P, coff);
    __syncthreads();
    using G = typename GeoSel<D, real>::T;
    const double dtd = S.dt;
    const real dt = (real)dtd;
    const real half = (real)0.5 * dt;
    const int i = i0 + (int)threadIdx.x / T;
    const int l = threadIdx.x % T;
    // moving walls: velocity rates at the sub-step's end (the level of v^{n+1}),
    // plus the given velocities
    const bool mv = MOVE && P.wmove, gv = MOVE && P.wvel;
    real Vw[3] = {0, 0, 0}, omw = 0;
    if (mv) wall_rates(P, ctrl->t + (S.tau + S.dt), Vw, omw);
    real speed = 0;
    uint32_t bad = 0;
    if (i < P.fbase + P.nf) {
        const R4<real> hi_ = hf[i];
        real vi[3];
        vi[0] = hi_.x; vi[1] = hi_.y;
        vi[2] = D == 3 ? hi_.z : (real)0;
        const real dev_i = D == 2 ? hi_.z : hi_.w;
        const real rho_i = P.rho0 + dev_i;
        const real p_i = P.c2 * dev_i;
        const real two_c = (real)2 * P.c, half_m = (real)0.5 * P.m;
        const G oi = geo[i];
        // the particle's own state for the final half-steps, loaded ahead of
        // the pair loop so that its latency hides behind it
        R4<real> so = {};
        double xo[3] = {0.0, 0.0, 0.0};
        constexpr bool ahead = D == 2 || SPHX_PREFETCH_3D;
        if (ahead && l == 0) {
            so = st[i];
            xo[0] = x0[i];
            xo[1] = x1[i];
            if (D == 3) xo[2] = x2[i];
        }
        real sum = 0;
        struct HalfJ { G o; R4<real> h; };
        struct WallJ { G o; G n; R4<real> k, g; };
        for_pairs<T, BATCH, T>(
            nbr, i, ncnt[i], P.maxn, l,
            [&](uint32_t e) {
                uint32_t j = e & NBR_MASK;
                HalfJ r;
                r.o = geo[j];
                r.h = hf[j];
                return r;
            },
            [&](uint32_t e, const HalfJ& r) {
                Pair<D, real> pq = pair_geo_c<D, real>(P, oi, r.o, coff[e >> NBR_SHIFT]);
                const R4<real>& hj = r.h;
                real dev_j = D == 2 ? hj.z : hj.w;
                // U_R - U_L = (v_j - v_i) . e_ij = (v_i - v_j) . d / r
                real dvd = (vi[0] - hj.x) * pq.d[0] + (vi[1] - hj.y) * pq.d[1] +
                           (D == 3 ? (vi[2] - hj.z) * pq.d[2] : (real)0);
                real rho_j = P.rho0 + dev_j;
                real inv_rho_j = div_r((real)1, rho_j);
                // U* - U_L = (U_R - U_L) / 2 + (p_i - p_j) / (2 rho_bar c) with
                // rho_bar = (rho_i + rho_j) / 2 and p = c^2 (rho - rho0):
                // 2 (U* - U_L) = (v_i - v_j) . d / r + 2 c (dev_i - dev_j) / (rho_i + rho_j)
                real dus2 = dvd * pq.rinv + div_r(two_c * (dev_i - dev_j), rho_i + rho_j);
                sum += half_m * inv_rho_j * dus2 * pq.dW;
            });
        for_pairs<T, BATCH, T>(
            wnb, i, wcnt[i], P.maxw, l,
            [&](uint32_t e) {
                uint32_t w = e & NBR_MASK;
                WallJ r;
                r.o = wgeo[w];
                r.n = wnrm[w];
                if (mv) r.k = wmot[w];
                if (gv) r.g = wvg[w];
                return r;
            },
            [&](uint32_t e, const WallJ& r) {
                Pair<D, real> pq = pair_geo_c<D, real>(P, oi, r.o, coff[e >> NBR_SHIFT]);
                const G& nw = r.n;
                real UL = -(nw.x * vi[0] + nw.y * vi[1] + (D == 3 ? zc(nw) * vi[2] : (real)0));
                // g . r_fw with r_fw = x_w - x_i = -d
                real gr = -(P.g[0] * pq.d[0] + P.g[1] * pq.d[1] + (D == 3 ? P.g[2] * pq.d[2] : (real)0));
                real pR = p_i + rho_i * gr;
                real rhoR = P.rho0 + pR * P.inv_c2;
                real rho_bar = (real)0.5 * (rho_i + rhoR);
                real us = div_r((p_i - pR) * P.half_inv_c, rho_bar);  // + (U_L + U_R)/2 = u_w below
                if (mv || gv) {
                    real vw[3] = {0, 0, 0};
                    if (mv) wall_velocity(r.k, Vw, omw, vw);
                    if (gv) add_given(r.g, vw);
                    us += -(nw.x * vw[0] + nw.y * vw[1] + (D == 3 ? zc(nw) * vw[2] : (real)0));
                }
                sum += P.vw * (us - UL) * pq.dW;
            });
        sum = group_sum<T>(sum);
        if (l == 0) {
            const real drho = (real)2 * rho_i * sum;
            if (!ahead) {
                so = st[i];
                xo[0] = x0[i];
                xo[1] = x1[i];
                if (D == 3) xo[2] = x2[i];
            }
            const double hd = 0.5 * dtd;
            xo[0] = xo[0] + hd * (double)so.x;
            xo[1] = xo[1] + hd * (double)so.y;
            if (D == 3) xo[2] = xo[2] + hd * (double)so.z;
            xo[0] = xo[0] + hd * (double)vi[0];
            xo[1] = xo[1] + hd * (double)vi[1];
            if (D == 3) xo[2] = xo[2] + hd * (double)vi[2];
            if (avt && P.p0 != (real)0) {
                // positions move with the transport velocity v + dt atv
                const R4<real> a = avt[2 * (size_t)i + 1];
                const double d2 = dtd * dtd;
                xo[0] = xo[0] + d2 * (double)a.x;
                xo[1] = xo[1] + d2 * (double)a.y;
                if (D == 3) xo[2] = xo[2] + d2 * (double)a.z;
            }
            x0[i] = xo[0];
            x1[i] = xo[1];
            if (D == 3) x2[i] = xo[2];
            R4<real> sn;
            sn.x = vi[0];
            sn.y = vi[1];
            if (D == 2) {
                sn.z = dev_i + half * drho;
                sn.w = drho;
            } else {
                sn.z = vi[2];
                sn.w = dev_i + half * drho;
                dr3[i] = drho;
                // and in w of the frozen offsets, where the pressure relaxation
                // gathers it with them (the pair loops here read x, y, z only)
                reinterpret_cast<real*>(const_cast<G*>(geo))[4 * (size_t)i + 3] = drho;
            }
            st[i] = sn;
            if (drho_out) drho_out[i] = drho;
            speed = sqrt(vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
            if (drho != drho || speed != speed) bad = ERR_NAN;
        }
    }
    if (bad) atomicOr(&ctrl->err_pending, bad);
    if (!finalize) return;
    // block maximum of |v^{n+1}| into the case's slots of this sub-step,
    // read by the next pressure relaxation or the step end (no cross-block
    // signalling here: a device-wide fence per block would write back L2)
    double m = wave_max((double)speed);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) smax[wid] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double bm = smax[0];
        for (int w = 1; w < pair_threads<T>() / 64; ++w) bm = fmax(bm, smax[w]);
        // relaxed, result unused: no wait, no fence; read after the kernel ends
        unsigned long long* vslot = vslot_all + (size_t)P.case_id * 2 * VSLOTS;
        atomicMax(&vslot[(q & 1) * VSLOTS + (b & (VSLOTS - 1))], speed_bits((real)bm));
    }
}

// (2D static: at most 64 VGPRs, eight wavefronts per SIMD; the kernel is
// latency-bound and the extra wavefront per SIMD pays)
template <int D, typename real, int T, bool MOVE>
__global__ __launch_bounds__(BLOCK) SPHX_PAIR_ATTR
__attribute__((amdgpu_waves_per_eu((D == 2 && !MOVE) ? 8 : 1))) void k_density(
    const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase, Ctrl* __restrict__ ctrl_all, int finalize,
    const typename GeoSel<D, real>::T* __restrict__ geo, const typename GeoSel<D, real>::T* __restrict__ wgeo,
    const typename GeoSel<D, real>::T* __restrict__ wnrm, const uint32_t* __restrict__ nbr,
    const int32_t* __restrict__ ncnt, const uint32_t* __restrict__ wnb, const int32_t* __restrict__ wcnt,
    const R4<real>* __restrict__ hf, R4<real>* __restrict__ st, real* __restrict__ dr3, double* __restrict__ x0,
    double* __restrict__ x1, double* __restrict__ x2, real* __restrict__ drho_out,
    unsigned long long* __restrict__ vslot_all, int q, const R4<real>* __restrict__ avt,
    const R4<real>* __restrict__ wmot, const R4<real>* __restrict__ wvg, int bin,
    const int32_t* __restrict__ cell, int32_t* __restrict__ key, int32_t* __restrict__ rank,
    int32_t* __restrict__ cnt)
{
    const int i0 = pair_block_first<T>(xcd_block(blockIdx.x, gridDim.x));
    bool static_code = !MOVE;
    if constexpr (MOVE) static_code = !wall_velocity_case(Pt, tcase, i0);
    // cases with static walls run the static instantiation's code
    if (static_code) {
        density_body<D, real, T, false>(
            Pt, tcase, ctrl_all, finalize, geo, wgeo, wnrm, nbr, ncnt, wnb, wcnt, hf, st, dr3, x0, x1, x2,
            drho_out, vslot_all, q, avt, wmot, wvg);
    } else {
        density_body<D, real, T, MOVE>(
            Pt, tcase, ctrl_all, finalize, geo, wgeo, wnrm, nbr, ncnt, wnb, wcnt, hf, st, dr3, x0, x1, x2,
            drho_out, vslot_all, q, avt, wmot, wvg);
    }
    if (!bin) return;
    // Last sub-step of a queue: the cell binning of the configuration update
    // (S1) for this block's slots, from the positions the block has just
    // written (every case, also one whose sub-steps are over), one
    // launch less per queue.
    __syncthreads();
    if (threadIdx.x >= 64) return;
    const KP<real>& P = Pt[tcase[i0 / TILE]];
    Ctrl* ctrl = ctrl_all + P.case_id;
    bin_slots<D>(P, ctrl, update_due(P, ctrl, 0, q), i0, pair_threads<T>() / T, x0, x1, x2, cell, key, rank, cnt);
}

// S5 after the last queued density relaxation, for case c, by one
// wavefront: close sub-step q. If the advection step is covered (or was
// covered earlier in the queue) prepare the next one; otherwise the step
// continues at the head of the next queue, its next sub-step stored in
// slot 0. Clears the case's |v| slots and folds the error bits the cell
// binning raised into the sticky ones.
template <typename real>
__device__ void step_end(const KP<real>& P, Ctrl* __restrict__ ctrl, unsigned long long* __restrict__ vslot, int q)
{
    const int lane = threadIdx.x & 63;
    const SubState Sp = ctrl->ss[q & 1];  // read by the whole wavefront before lane 0 writes
    const uint32_t err = ctrl->err;
    bool cont = false;
    if (Sp.active && !err) {
        const double vmax = slot_max<real>(vslot + (q & 1) * VSLOTS);
        bool finished;
        SubState n = next_substep(P, ctrl->dt_ad, Sp, vmax, finished);
        cont = !finished;
        if (lane == 0) close_substep(ctrl, 0, n, vmax, finished);
    }
    vslot[lane] = 0ull;
    vslot[VSLOTS + lane] = 0ull;
    if (lane != 0) return;
    const uint32_t pend = ctrl->err_pending;
    if (pend) {
        ctrl->err_pending = 0u;
        ctrl->err |= pend;
    }
    if (err || ctrl->err) return;
    if (cont) {
        ctrl->ss[1].active = 0;
        ctrl->midstep = 1;
    } else {
        prepare_step(P, ctrl);
    }
}

// Whether the configuration update at the end of a queue is a full one for
// this case: requested, an advection step ended earlier in the queue, or the
// last queued sub-step q (q >= 0) ends it. The same decision as step_end's
// (next_substep's `finished`, which does not depend on |v|max), taken from
// the same state by every wavefront, also inside the density relaxation of
// sub-step q itself (nothing it writes enters the decision).
template <typename real>
__device__ __forceinline__ bool update_due(const KP<real>& P, const Ctrl* __restrict__ ctrl, int force, int q)
{
    if (force || ctrl->rebuild) return true;
    if (q < 0) return false;
    const SubState Sp = ctrl->ss[q & 1];
    if (!Sp.active || ctrl->err) return false;
    return Sp.last || !(ctrl->dt_ad - (Sp.tau + Sp.dt) > 0.0);
}

// Single-pass exclusive scan of the cell counts (decoupled look-back), for
// grids of at most LB_MAX_BLOCKS tiles, where every block finds all its
// predecessors in one window (no chain of waits): each
// block takes a ticket (its tile, in the order blocks start), reduces its
// tile, publishes the aggregate, then adds the aggregates and prefixes of
// the tiles before it as they appear and publishes its own inclusive prefix.
// A block only waits for tiles with smaller tickets, whose blocks are
// already running, so every wait ends; a bounded spin records a fault in
// *fault instead of waiting for ever. Status words carry an epoch, so no
// clearing is needed between scans: the last ticket's block advances the
// epoch and resets the ticket counter. The counts are consumed (zeroed).
// With q >= 0 the blocks also run step_end for every case (cases spread
// over the wavefronts of the grid).
constexpr uint32_t LB_AGG = 1u, LB_PREFIX = 2u;
constexpr int LB_SPIN_CAP = 1 << 22;
constexpr int LB_ITEMS = 8;                   // consecutive counts per thread
constexpr int LB_TILE = BLOCK * LB_ITEMS;     // counts per block
constexpr int LB_MAX_BLOCKS = 64;             // grids up to one look-back window use the single pass

template <typename real>
__global__ __launch_bounds__(BLOCK) void k_scan_lb(int32_t* __restrict__ cnt, int32_t* __restrict__ start, int n,
                                                   unsigned long long* __restrict__ status, int32_t* __restrict__ ticket,
                                                   uint32_t* __restrict__ epoch, int32_t* __restrict__ fault,
                                                   const KP<real>* __restrict__ Pt, Ctrl* __restrict__ ctrl_all,
                                                   unsigned long long* __restrict__ vslot_all, int q, int ncase)
{
    __shared__ int sh[BLOCK];
    __shared__ int s_ticket, s_excl;
    __shared__ uint32_t s_epoch;
    if (threadIdx.x == 0) {
        s_epoch = __hip_atomic_load(epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_ticket = atomicAdd(ticket, 1);
    }
    __syncthreads();
    const int b = s_ticket;
    const uint32_t ep = s_epoch;
    const int nb = gridDim.x;
    const int base = b * LB_TILE + threadIdx.x * LB_ITEMS;
    int v[LB_ITEMS];
    int sum = 0;
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
        v[k] = base + k < n ? cnt[base + k] : 0;
        sum += v[k];
    }
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k)
        if (base + k < n) cnt[base + k] = 0;
    int total;
    int ex = block_excl_scan(sum, sh, total);
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const unsigned long long tag_agg = (unsigned long long)((ep << 2) | LB_AGG) << 32;
        const unsigned long long tag_pre = (unsigned long long)((ep << 2) | LB_PREFIX) << 32;
        int excl = 0;
        if (b > 0) {
            if (lane == 0)
                __hip_atomic_store(&status[b], tag_agg | (uint32_t)total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // windows of 64 predecessors, nearest first, until one has a prefix
            for (int j = b - 1; j >= 0; j -= 64) {
                const int k = j - lane;
                unsigned long long w = 0ull;
                bool pre = false;
                int val = 0;
                if (k >= 0) {
                    for (int it = 0;; ++it) {
                        w = __hip_atomic_load(&status[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const unsigned long long tag = w & 0xffffffff00000000ull;
                        if (tag == tag_agg || tag == tag_pre) break;
                        if (it >= LB_SPIN_CAP) {
                            atomicOr(fault, 1);
                            w = tag_pre;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    pre = (w & 0xffffffff00000000ull) == tag_pre;
                    val = (int)(uint32_t)w;
                }
                const unsigned long long pm = __ballot(pre);
                const int stop = pm ? __ffsll((long long)pm) - 1 : 64;
                int c = (k >= 0 && lane <= stop) ? val : 0;
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
                excl += c;
                if (pm) break;
            }
        }
        if (lane == 0) {
            __hip_atomic_store(&status[b], tag_pre | (uint32_t)(excl + total), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            s_excl = excl;
        }
    }
    __syncthreads();
    ex += s_excl;
#pragma unroll
    for (int k = 0; k < LB_ITEMS; ++k) {
        if (base + k < n) start[base + k] = ex;
        ex += v[k];
    }
    if (b == nb - 1 && threadIdx.x == 0) {
        start[n] = s_excl + total;
        __hip_atomic_store(ticket, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(epoch, ep == 0x3fffffffu ? 1u : ep + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (q < 0) return;
    const int waves = BLOCK / 64, wid = threadIdx.x / 64;
    for (int c = b * waves + wid; c < ncase; c += nb * waves)
        step_end(Pt[c], ctrl_all + c, vslot_all + (size_t)c * 2 * VSLOTS, q);
}

// Second pass of the two-pass scan used for larger grids (after
// k_scan_tiles): each block adds the sum of the tile sums before it (read
// directly, no scan of the sums) to its tile; the last block writes the
// total. With q >= 0 the blocks also run step_end for every case.
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_scan_fin(int32_t* __restrict__ start, const int32_t* __restrict__ bsum,
                                                    int n, const KP<real>* __restrict__ Pt,
                                                    Ctrl* __restrict__ ctrl_all,
                                                    unsigned long long* __restrict__ vslot_all, int q, int ncase)
{
    __shared__ int sh[BLOCK];
    const int b = blockIdx.x, nb = gridDim.x;
    int s = 0;
    for (int k = threadIdx.x; k < b; k += BLOCK) s += bsum[k];
    int before;
    (void)block_excl_scan(s, sh, before);
    const int base = b * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k)
        if (base + k < n) start[base + k] += before;
    if (b == nb - 1 && threadIdx.x == 0) start[n] = before + bsum[b];
    if (q < 0) return;
    const int waves = BLOCK / 64, wid = threadIdx.x / 64;
    for (int c = b * waves + wid; c < ncase; c += nb * waves)
        step_end(Pt[c], ctrl_all + c, vslot_all + (size_t)c * 2 * VSLOTS, q);
}

// ---------------------------------------------------------------------
// |v|max of the current state of every case (only < 0) or of case `only`,
// restricted to the cases with mask[c] != 0 if a mask is given (outside the
// time loop; one thread per slot).
template <int D, typename real>
__global__ __launch_bounds__(BLOCK) void k_vmax(const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase,
                                                int ntiles, int only, const int32_t* __restrict__ mask,
                                                Ctrl* __restrict__ ctrl_all, const R4<real>* __restrict__ st)
{
    const int tile = wave_tile();
    if (tile >= ntiles) return;
    const KP<real>& P = Pt[tcase[tile]];
    if ((only >= 0 && P.case_id != only) || (mask && !mask[P.case_id])) return;
    const int i = tile * TILE + (threadIdx.x & 63);
    real sp = 0;
    if (i < P.fbase + P.nf) {
        R4<real> s = st[i];
        sp = D == 2 ? sqrt(s.x * s.x + s.y * s.y) : sqrt(s.x * s.x + s.y * s.y + s.z * s.z);
    }
    double m = wave_max((double)sp);
    if ((threadIdx.x & 63) == 0) atomicMax(&ctrl_all[P.case_id].vmax_bits, speed_bits((real)m));
}

template <typename real>
__global__ void k_vmax_fin(Ctrl* __restrict__ ctrl_all, int ncases, int only, const int32_t* __restrict__ mask)
{
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncases || (only >= 0 && c != only) || (mask && !mask[c])) return;
    ctrl_all[c].vmax = bits_speed<real>(ctrl_all[c].vmax_bits);
    ctrl_all[c].vmax_bits = 0ull;
}

// ---------------------------------------------------------------------
// S8: FP64 diagnostics. Per tile partial sums; k_diag_fin reduces each
// case's tiles in a fixed order so the result is deterministic.
constexpr int NDIAG = 8;  // mom0..2, e_kin, e_pot, e_int, front (max), max |dev|/rho0 (max)

template <int D, typename real>
__global__ __launch_bounds__(BLOCK) void k_diag(const KP<real>* __restrict__ Pt, const int32_t* __restrict__ tcase,
                                                int ntiles, const double* __restrict__ x0,
                                                const double* __restrict__ x1, const double* __restrict__ x2,
                                                const R4<real>* __restrict__ st, double* __restrict__ part)
{
    const int tile = wave_tile();
    if (tile >= ntiles) return;
    const KP<real>& P = Pt[tcase[tile]];
    const int lane = threadIdx.x & 63;
    const int i = tile * TILE + lane;
    double v[NDIAG] = {0, 0, 0, 0, 0, 0, -1e300, 0};
    if (i < P.fbase + P.nf) {
        R4<real> s = st[i];
        double m = P.md;
        double vel[3] = {(double)s.x, (double)s.y, D == 3 ? (double)s.z : 0.0};
        double dev = D == 2 ? (double)s.z : (double)s.w;
        double x[3] = {x0[i], x1[i], D == 3 ? x2[i] : 0.0};
        v[0] = m * vel[0];
        v[1] = m * vel[1];
        v[2] = m * vel[2];
        v[3] = 0.5 * m * (vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]);
        v[4] = -m * ((double)P.g[0] * x[0] + (double)P.g[1] * x[1] + (double)P.g[2] * x[2]);
        double a = dev / P.rho0d;                 // rho/rho0 - 1
        v[5] = m * (double)P.c0d * P.c0d * (log1p(a) - a / (1.0 + a));
        v[6] = x[0];
        v[7] = fabs(a);
    }
#pragma unroll
    for (int q = 0; q < NDIAG; ++q) {
        double r = (q == 6 || q == 7) ? wave_max(v[q]) : wave_sum(v[q]);
        if (lane == 0) part[(size_t)tile * NDIAG + q] = r;
    }
}

// One block per case, fixed reduction order (strided partials, then
// shuffle trees), so the result does not depend on timing.
template <typename real>
__global__ __launch_bounds__(BLOCK) void k_diag_fin(const KP<real>* __restrict__ Pt, const double* __restrict__ part,
                                                    double* __restrict__ out)
{
    const KP<real>& P = Pt[blockIdx.x];
    const int t0 = P.fbase / TILE, nt = P.fcap / TILE;
    __shared__ double sh[NDIAG][BLOCK / 64];
    double v[NDIAG];
#pragma unroll
    for (int q = 0; q < NDIAG; ++q) v[q] = q == 6 ? -1e300 : 0.0;
    for (int b = threadIdx.x; b < nt; b += BLOCK)
#pragma unroll
        for (int q = 0; q < NDIAG; ++q) {
            double x = part[(size_t)(t0 + b) * NDIAG + q];
            v[q] = (q == 6 || q == 7) ? fmax(v[q], x) : v[q] + x;
        }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NDIAG; ++q) {
        double r = (q == 6 || q == 7) ? wave_max(v[q]) : wave_sum(v[q]);
        if (lane == 0) sh[q][wid] = r;
    }
    __syncthreads();
    if (threadIdx.x < NDIAG) {
        int q = threadIdx.x;
        double r = sh[q][0];
        for (int w = 1; w < BLOCK / 64; ++w) r = (q == 6 || q == 7) ? fmax(r, sh[q][w]) : r + sh[q][w];
        out[(size_t)blockIdx.x * NDIAG + q] = r;
    }
}

// ---------------------------------------------------------------------
// Output helpers: one case's field back to its original order, as FP64.
template <int D, typename real>
__global__ __launch_bounds__(BLOCK) void k_unsort_field(const KP<real>* __restrict__ Pt, int c, int which,
                                                        const int32_t* __restrict__ id, const double* __restrict__ x0,
                                                        const double* __restrict__ x1, const double* __restrict__ x2,
                                                        const R4<real>* __restrict__ st, const real* __restrict__ dr3,
                                                        double* __restrict__ out)
{
    const KP<real>& P = Pt[c];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.nf) return;
    const int i = P.fbase + k;
    const int o = id[i];
    R4<real> s = st[i];
    double dev = D == 2 ? (double)s.z : (double)s.w;
    switch (which) {
    case 0:
        out[(size_t)o * D + 0] = x0[i];
        out[(size_t)o * D + 1] = x1[i];
        if (D == 3) out[(size_t)o * D + 2] = x2[i];
        break;
    case 1:
        out[(size_t)o * D + 0] = (double)s.x;
        out[(size_t)o * D + 1] = (double)s.y;
        if (D == 3) out[(size_t)o * D + 2] = (double)s.z;
        break;
    case 2: out[o] = P.rho0d + dev; break;
    case 3: out[o] = (double)P.c0d * P.c0d * dev; break;
    case 4: out[o] = D == 2 ? (double)s.w : (double)dr3[i]; break;
    default: break;
    }
}

template <typename real>
__global__ __launch_bounds__(BLOCK) void k_unsort_vec(int base, int n, int width, const int32_t* __restrict__ id,
                                                      const real* __restrict__ in, double* __restrict__ out)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int i = base + k;
    const int o = id[i];
    for (int w = 0; w < width; ++w) out[(size_t)o * width + w] = (double)in[(size_t)i * width + w];
}

// Load one case's particles, given in original order, into its slots.
template <int D, typename real>
__global__ __launch_bounds__(BLOCK) void k_load_fluid(const KP<real>* __restrict__ Pt, int c,
                                                      const double* __restrict__ pos, const double* __restrict__ vel,
                                                      const double* __restrict__ rho, const double* __restrict__ drho,
                                                      double* __restrict__ x0, double* __restrict__ x1,
                                                      double* __restrict__ x2, R4<real>* __restrict__ st,
                                                      real* __restrict__ dr3, int32_t* __restrict__ id,
                                                      int32_t* __restrict__ cell)
{
    const KP<real>& P = Pt[c];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.nf) return;
    const int i = P.fbase + k;
    x0[i] = pos[(size_t)k * D + 0];
    x1[i] = pos[(size_t)k * D + 1];
    if (D == 3) x2[i] = pos[(size_t)k * D + 2];
    double v[3] = {0, 0, 0};
    if (vel)
        for (int a = 0; a < D; ++a) v[a] = vel[(size_t)k * D + a];
    double dev = rho ? rho[k] - P.rho0d : 0.0;
    double dr = drho ? drho[k] : 0.0;
    R4<real> s;
    s.x = (real)v[0];
    s.y = (real)v[1];
    if (D == 2) {
        s.z = (real)dev;
        s.w = (real)dr;
    } else {
        s.z = (real)v[2];
        s.w = (real)dev;
        dr3[i] = (real)dr;
    }
    st[i] = s;
    id[i] = k;
    cell[i] = P.cbase;  // replaced by the next (full) binning
}

}  // namespace sphx
