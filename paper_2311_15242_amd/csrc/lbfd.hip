// lbfd.hip -- MI355X (gfx950) solver for the hybrid lattice-Boltzmann
// colour-gradient / finite-difference method for two-phase flow with soluble
// surfactants (Ba, Liu, Li, Yang; arXiv 2311.15242), behind the C ABI of lbfd.h.
//
// Per time step n -> n+1 the stream carries:
//   collide  MRT collision with correction and forcing terms (eqs 1-4, App. A),
//            recolouring descriptor (eqs 11-12), push propagation with
//            half-way bounce-back (eq 13)
//   macro    rho^R, rho^B, rhoN (eq 6) and momentum of step n+1
//   geom     |grad rhoN| and the normal at n+1 (below eq 6)
//   fd       WENO3 convection (eqs 25-27), sources (eq 22), explicit half of
//            the diffusion (eq 28) and the Crank-Nicolson right-hand sides
//            (eqs 23-24)
//   sor      red-black SOR sweeps of the two implicit systems (Sec 2.2)
//   total    FP64 deterministic sum of the conserved surfactant and the
//            rescaling factor (applied lazily by every later reader)
//   force    curvature (eq 7), equation of state (eq 8), interfacial force
//            (eq 9), buoyancy (Sec 3.4) and velocity (eq 10) of step n+1
#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <vector>

#include "lbfd.h"
#include "lbfd_kernels.h"
#include "lbfd_surrogate.h"
#include "sg_conv.h"

namespace lbfd {

constexpr int BX = 64, BY = 4;          // one wavefront spans 64 consecutive x
static_assert(BX == 64, "node kernels hold y in scalar registers: a wavefront must be one row");
constexpr int NRED = 19;                 // observable partial sums per block
constexpr int TOTAL_BLOCKS = 1024;       // most workgroups of the total-surfactant sum
constexpr int TOTAL_NODES = 4096;        // nodes per workgroup of that sum below the cap

// Workgroups of the total-surfactant sum of an N-node grid. A function of N
// alone, so the summation order (and the rounded total) of an instance is the
// same whether it is stepped alone or in a batch.
inline int total_blocks(long long N)
{
    const long long b = (N + TOTAL_NODES - 1) / TOTAL_NODES;
    return (int)(b < 1 ? 1 : b > TOTAL_BLOCKS ? TOTAL_BLOCKS : b);
}

struct InitDev {
    int n;
    double cx[16], cy[16], cz[16], r[16];
    double width, psi0, phi0_out, phi0_in, shear_rate;
};

// ============================================================== initial state

// Colour field and per-colour equilibria of the initial state at one node.
template <int LAT, class R>
__device__ void init_node(const KP<R> &k, const InitDev &in, int x, int y, int z, R &rN, R *fR, R *fB, R *u0)
{
    using L = Lat<LAT>;
    double best = -1.0;
    for (int d = 0; d < in.n; ++d) {
        double dx = x - in.cx[d], dy = y - in.cy[d], dz = L::D == 3 ? z - in.cz[d] : 0.0;
        double v = tanh(2.0 * (in.r[d] - sqrt(dx * dx + dy * dy + dz * dz)) / in.width);
        if (d == 0 || v > best) best = v;
    }
    rN = (R)best;
    R rR = k.rhoR0 * (R(1) + rN) / R(2), rB = k.rhoB0 * (R(1) - rN) / R(2);
    u0[0] = (R)(in.shear_rate * (y - 0.5 * (k.ny - 1)));
    u0[1] = 0;
    u0[2] = 0;
    // f^k = M^-1 m^{k,eq}(rho^k, alpha^k, u0): the moments below are eq 37 / eq 40
    for (int c = 0; c < 2; ++c) {
        R rho = c == 0 ? rR : rB, m[QMAX];
        R al = k.alpha[c];
        R ux = u0[0], uy = u0[1], uz = u0[2], u2 = ux * ux + uy * uy + uz * uz;
        if constexpr (L::D == 2) {
            m[0] = rho; m[1] = rho * (R(-3.6) * al - R(0.4) + R(3) * u2); m[2] = rho * (R(5.4) * al - R(1.4) - R(3) * u2);
            m[3] = rho * ux; m[4] = rho * (R(-1.8) * al - R(0.2)) * ux; m[5] = rho * uy;
            m[6] = rho * (R(-1.8) * al - R(0.2)) * uy; m[7] = rho * (ux * ux - uy * uy); m[8] = rho * ux * uy;
        } else {
            R pk = rho * k.cs2[c];
            m[0] = rho; m[1] = rho * ux; m[2] = rho * uy; m[3] = rho * uz; m[4] = R(3) * pk + rho * u2;
            m[5] = rho * (R(2) * ux * ux - uy * uy - uz * uz); m[6] = rho * (uy * uy - uz * uz);
            m[7] = rho * ux * uy; m[8] = rho * ux * uz; m[9] = rho * uy * uz;
            m[10] = pk * uy; m[11] = pk * ux; m[12] = pk * uz; m[13] = pk * ux; m[14] = pk * uz; m[15] = pk * uy;
            R b = R(1) - al - u2;
            m[16] = rho * (b + R(2) * (ux * ux + uy * uy)) / R(6);
            m[17] = rho * (b + R(2) * (ux * ux + uz * uz)) / R(6);
            m[18] = rho * (b + R(2) * (uy * uy + uz * uz)) / R(6);
        }
        R *out = c == 0 ? fR : fB;
        for (int i = 0; i < L::Q; ++i) {
            R a = 0;
            for (int r = 0; r < L::Q; ++r) a += R(L::MINV[i][r]) * m[r];
            out[i] = a;
        }
    }
}

// Sum over colours of the moment equilibria m^{k,eq}(rho^k, alpha^k, u), eq 37 (2-D) / eq 40 (3-D).
template <int LAT, class R> __device__ __forceinline__ void meq_sum(const KP<R> &k, R rR, R rB, const R *u, R *meq)
{
    using L = Lat<LAT>;
    constexpr int D = L::D;
#pragma unroll
    for (int r = 0; r < L::Q; ++r) meq[r] = 0;
    const R ux = u[0], uy = u[1], uz = D == 3 ? u[2] : R(0), u2 = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const R rk = c == 0 ? rR : rB;
        const R al = k.alpha[c];
        if constexpr (D == 2) {
            meq[0] += rk; meq[1] += rk * (R(-3.6) * al - R(0.4) + R(3) * u2);
            meq[2] += rk * (R(5.4) * al - R(1.4) - R(3) * u2);
            meq[3] += rk * ux; meq[4] += rk * (R(-1.8) * al - R(0.2)) * ux;
            meq[5] += rk * uy; meq[6] += rk * (R(-1.8) * al - R(0.2)) * uy;
            meq[7] += rk * (ux * ux - uy * uy); meq[8] += rk * ux * uy;
        } else {
            const R pc = rk * k.cs2[c];
            meq[0] += rk; meq[1] += rk * ux; meq[2] += rk * uy; meq[3] += rk * uz;
            meq[4] += R(3) * pc + rk * u2; meq[5] += rk * (R(2) * ux * ux - uy * uy - uz * uz);
            meq[6] += rk * (uy * uy - uz * uz); meq[7] += rk * ux * uy; meq[8] += rk * ux * uz;
            meq[9] += rk * uy * uz; meq[10] += pc * uy; meq[11] += pc * ux; meq[12] += pc * uz;
            meq[13] += pc * ux; meq[14] += pc * uz; meq[15] += pc * uy;
            const R b = R(1) - al - u2;
            const R r6 = rk * R(1.0 / 6.0);
            meq[16] += r6 * (b + R(2) * (ux * ux + uy * uy));
            meq[17] += r6 * (b + R(2) * (ux * ux + uz * uz));
            meq[18] += r6 * (b + R(2) * (uy * uy + uz * uz));
        }
    }
}

// State between steps in the deviation modes: the moments m = M f of each
// node, stored as their difference from a node-local reference, the summed
// equilibrium moments at the node's own rho^R, rho^B and u = j / rho. The
// conserved rows (mass, momentum) equal their reference and are not stored;
// the others are stored in 16 bits, compacted to the first Q - 1 - D planes
// of the population buffer.
template <int LAT, class P>
__device__ __forceinline__ void load_moments(const KP<typename P::R> &k, const typename P::S *fs, uint32_t n,
                                             typename P::R rR, typename P::R rB, const typename P::R *uj,
                                             typename P::R *m)
{
    using R = typename P::R;
    using L = Lat<LAT>;
    meq_sum<LAT, R>(k, rR, rB, uj, m);
#pragma unroll
    for (int r = 0; r < L::Q; ++r)
        if (!conserved_row<LAT>(r)) m[r] += to_real(ldu(fs + (long long)state_slot<LAT>(r) * k.N, n));
}

template <int LAT, class P>
__device__ __forceinline__ void store_moments(const KP<typename P::R> &k, typename P::S *fs, uint32_t n,
                                              typename P::R rR, typename P::R rB, const typename P::R *uj,
                                              const typename P::R *m, Dither *dz = nullptr)
{
    using R = typename P::R;
    using S = typename P::S;
    using L = Lat<LAT>;
    R mref[L::Q];
    meq_sum<LAT, R>(k, rR, rB, uj, mref);
#pragma unroll
    for (int r = 0; r < L::Q; ++r)
        if (!conserved_row<LAT>(r)) {
            const R v = m[r] - mref[r];
            stu(fs + (long long)state_slot<LAT>(r) * k.N, n, dz ? from_real_sr<S>(v, dz->next()) : from_real<S>(v));
        }
}

// Store the populations f of node n at the start of a step: as populations,
// or in the deviation modes as moments (above).
template <int LAT, class P>
__device__ __forceinline__ void store_state(const KP<typename P::R> &k, typename P::S *fo, long long n, const typename P::R *f,
                                            typename P::R rR, typename P::R rB, const typename P::R *j)
{
    using R = typename P::R;
    using L = Lat<LAT>;
    constexpr int Q = L::Q;
    if constexpr (P::DEV) {
        R m[Q], uj[3] = {0, 0, 0};
#pragma unroll
        for (int r = 0; r < Q; ++r) {
            m[r] = 0;
#pragma unroll
            for (int i = 0; i < Q; ++i)
                if (L::M[r][i] != 0) m[r] += R(L::M[r][i]) * f[i];
        }
#pragma unroll
        for (int d = 0; d < L::D; ++d) uj[d] = j[d] / (rR + rB);
        store_moments<LAT, P>(k, fo, n, rR, rB, uj, m);
    } else {
#pragma unroll
        for (int i = 0; i < Q; ++i) fo[(long long)i * k.N + n] = f[i];
    }
}

template <int LAT, class P> __global__ __launch_bounds__(256) void k_init(KP<typename P::R> k, InitDev in)
{
    using R = typename P::R;
    using S = typename P::S;
    using L = Lat<LAT>;
    Node nd = node_id(k);
    if (!nd.ok) return;
    const long long N = k.N, n = lin(k, nd.x, nd.y, nd.z);
    R rN0, fR[QMAX], fB[QMAX], u0[3], f[QMAX];
    init_node<LAT, R>(k, in, nd.x, nd.y, nd.z, rN0, fR, fB, u0);
    R rR = 0, rB = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < L::Q; ++i) {
        rR += fR[i];
        rB += fB[i];
        f[i] = fR[i] + fB[i];
        for (int d = 0; d < L::D; ++d) j[d] += f[i] * R(L::E[i][d]);
    }
    R rr = rR / k.rhoR0, bb = rB / k.rhoB0;
    R *mac = k.fld.mac[k.lev];
    mac[n] = rR;
    mac[N + n] = rB;
    mac[2 * N + n] = (rr - bb) / (rr + bb);
    for (int d = 0; d < L::D; ++d) mac[(3 + d) * N + n] = j[d];
    store_state<LAT, P>(k, (S *)k.fld.f[k.fc], n, f, rR, rB, j);
    k.fld.psi[k.pc][n] = (R)in.psi0;
    k.fld.phi[k.pc][n] = rN0 < R(0) ? (R)in.phi0_out : (R)in.phi0_in;
    k.fld.Sp[n] = 0;
    k.fld.Bp[n] = 0;
}

// State import from FP64 arrays (device copies).
template <int LAT, class P>
__global__ __launch_bounds__(256) void k_import(KP<typename P::R> k, const double *f_, const double *rR_,
                                               const double *rB_, const double *psi, const double *phi,
                                               const double *Sp, const double *Bp)
{
    using R = typename P::R;
    using S = typename P::S;
    using L = Lat<LAT>;
    Node nd = node_id(k);
    if (!nd.ok) return;
    const long long N = k.N, n = lin(k, nd.x, nd.y, nd.z);
    R rR = (R)rR_[n], rB = (R)rB_[n], j[3] = {0, 0, 0}, f[QMAX];
    for (int i = 0; i < L::Q; ++i) {
        f[i] = (R)f_[i * N + n];
        for (int d = 0; d < L::D; ++d) j[d] += f[i] * R(L::E[i][d]);
    }
    R rr = rR / k.rhoR0, bb = rB / k.rhoB0;
    R *mac = k.fld.mac[k.lev];
    mac[n] = rR;
    mac[N + n] = rB;
    mac[2 * N + n] = (rr - bb) / (rr + bb);
    for (int d = 0; d < L::D; ++d) mac[(3 + d) * N + n] = j[d];
    store_state<LAT, P>(k, (S *)k.fld.f[k.fc], n, f, rR, rB, j);
    k.fld.psi[k.pc][n] = (R)psi[n];
    k.fld.phi[k.pc][n] = (R)phi[n];
    k.fld.Sp[n] = Sp ? (R)Sp[n] : R(0);
    k.fld.Bp[n] = Bp ? (R)Bp[n] : R(0);
}

// ============================================================== LDS halos

// A 64 x TY node tile (one plane) and its one-node halo: 66 x (TY + 2) (x 3 planes
// in 3-D).
template <int D, int TY> struct Halo1 {
    static constexpr int HX = BX + 2, HY = TY + 2, HZ = D == 3 ? 3 : 1, HN = HX * HY * HZ;
    static constexpr int HS = (HN + BX * TY - 1) / (BX * TY);   // cells per thread
    // halo cell of the thread's own node
    __device__ static int self() { return (int)(threadIdx.x + 1) + HX * ((int)(threadIdx.y + 1) + HY * (D == 3 ? 1 : 0)); }
    // offset of the neighbour at lattice offset (ex, ey, ez)
    __host__ __device__ static constexpr int off(int ex, int ey, int ez) { return ex + HX * (ey + HY * ez); }
};

// Halo coordinate along one axis: wrapped on a periodic axis, the mirror node
// beyond a wall (what the lattice stencils read there); cells that no node of
// the tile reads are clamped into the grid.
__device__ __forceinline__ int halo_coord(int g, int n, int wall)
{
    if (g >= 0 && g < n) return g;
    if (wall) {
        g = g < 0 ? -1 - g : 2 * n - 1 - g;
        return g < 0 ? 0 : (g >= n ? n - 1 : g);
    }
    if (g < 0) g += n;
    while (g >= n) g -= n;
    return g;
}

// Stage NF node arrays of a tile and its one-node halo in LDS, a row of HX cells
// per wavefront at a time: each lane holds one x column (lanes 0 and 1 a second
// one), whose wrap is worked out once; the rows' y and z are uniform. Every
// wavefront issues all of its loads before its LDS stores. The caller
// synchronises the workgroup before reading.
template <int LAT, class T, int NF, int TY, class R>
__device__ __forceinline__ void stage_halo1(const KP<R> &k, int tile, const T *const *src,
                                            T (*sh)[Halo1<Lat<LAT>::D, TY>::HN])
{
    constexpr int D = Lat<LAT>::D;
    using H = Halo1<D, TY>;
    constexpr int NR = H::HY * H::HZ, RPW = (NR + TY - 1) / TY;   // rows, rows per wavefront
    const int bx = tile % k.gx, rr = tile / k.gx, gy = gy_of(k, TY);
    const int ox = bx * BX - 1, oy = (rr % gy) * TY - 1, oz = rr / gy - (D == 3 ? 1 : 0);
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int lane = (int)threadIdx.x;
    const bool two = lane < H::HX - BX;
    const uint32_t gx0 = (uint32_t)halo_coord(ox + lane, k.nx, k.bc[0]);
    const uint32_t gx1 = two ? (uint32_t)halo_coord(ox + BX + lane, k.nx, k.bc[0]) : 0u;
    T v0[RPW][NF], v1[RPW][NF];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int row = w + TY * i;
        if (row >= NR) continue;
        const int gy = halo_coord(oy + row % H::HY, k.ny, k.bc[1]);
        const int gz = D == 3 ? halo_coord(oz + row / H::HY, k.nz, k.bc[2]) : 0;
        const uint32_t base = (uint32_t)k.nx * ((uint32_t)gy + (uint32_t)k.ny * (uint32_t)gz);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            v0[i][f] = ldu(src[f], base + gx0);
            if (two) v1[i][f] = ldu(src[f], base + gx1);
        }
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
        const int row = w + TY * i;
        if (row >= NR) continue;
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            sh[f][row * H::HX + lane] = v0[i][f];
            if (two) sh[f][row * H::HX + BX + lane] = v1[i][f];
        }
    }
}

// lat_deriv on a staged field: the same stencil, pairs and mirror signs.
template <int LAT, int TY, class R>
__device__ __forceinline__ R lat_deriv_lds(const Nbhd &b, const R *sh, int hself, R scl, int a, int odd_axis)
{
    using L = Lat<LAT>;
    using H = Halo1<L::D, TY>;
    R acc = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        if (L::OPP[i] < i || L::E[i][a] == 0) continue;
        const int ex = L::E[i][0], ey = L::E[i][1], ez = L::E[i][2];
        R vp = sh[hself + H::off(ex, ey, ez)];
        R vm = sh[hself - H::off(ex, ey, ez)];
        if (odd_axis >= 0) {
            const int eo = L::E[i][odd_axis];
            if (nb_wall_axis(b, odd_axis, eo)) vp = -vp;
            if (nb_wall_axis(b, odd_axis, -eo)) vm = -vm;
        }
        acc += R(L::W[i] * L::E[i][a]) * (vp - vm);
    }
    return R(3) * acc * scl;
}

// ============================================================== geometry

// |grad rhoN| and the regularised normal n = -grad rhoN / sqrt(|grad rhoN|^2 + eps^2)
// of the time level `level` (below eq 6).
template <int LAT, class P> __device__ __forceinline__ void geom_body(const KP<typename P::R> &k, int tile, const StepArgs &sa, int level)
{
    using R = typename P::R;
    using L = Lat<LAT>;
    // one geometry launch per step: it advances the step counter of the stochastic
    // rounding, which only the collision and macro kernels (earlier in the step) read
    if constexpr (P::DEV)
        if (tile == 0 && threadIdx.x == 0 && threadIdx.y == 0) k.fld.sc->tick += 1u;
    Node nd = node_at(k, tile);
    if (!nd.ok) return;
    const long long N = k.N;
    const uint32_t n = node_index(k, nd);
    const R *rN = k.fld.mac[level] + 2 * N;
    const Nbhd nb = make_nbhd(k, nd.x, nd.y, nd.z);
    R g[3], G2 = 0;
#pragma unroll
    for (int a = 0; a < L::D; ++a) {
        g[a] = lat_deriv<LAT, R>(nb, rN, n, R(1), a, -1);
        G2 += g[a] * g[a];
    }
    const R G = sqrt(G2);
    st(k.fld.G[level], n, G);
    R den = sqrt(G2 + k.eps_n * k.eps_n);
#pragma unroll
    for (int a = 0; a < L::D; ++a) st(k.fld.nrm + a * N, n, den > R(0) ? -g[a] / den : R(0));
    // node weights of the implicit systems at this level, W = G + eps (psi) and
    // X + eps = 1 - rhoN + eps (phi), in the solve's colour-split arrays: the level
    // a geometry launch computes is always the one the next solve needs
    const uint32_t j = split_idx(k, nd.x, nd.y, nd.z);
    st(k.fld.cw2, j, V2<R>{G + k.fd_eps, (R(1) - ld(rN, n)) + k.fd_eps});
}
template <int LAT, class P> __global__ __launch_bounds__(256) void k_geom(KP<typename P::R> k, int level)
{
    geom_body<LAT, P>(k, xcd_tile((int)blockIdx.x, (int)gridDim.x), step_args(k), level);
}
template <int LAT, class P>
__global__ __launch_bounds__(256) void kb_geom(const KP<typename P::R> *tab, const int *prefix, int ninst, StepArgs sa, int level)
{
    int inst, local;
    batch_tile(prefix, ninst, inst, local);
    geom_body<LAT, P>(tab[inst], local, sa, level);
}

// ============================================================== forces

// Curvature (eq 7), modified Langmuir EOS (eq 8), interfacial force with the
// Marangoni term (eq 9), buoyancy (Sec 3.4), total force and velocity (eq 10)
// at the current time level.
template <int LAT, class P, int TY>
__device__ __forceinline__ void force_body(const KP<typename P::R> &k, int tile, const StepArgs &sa)
{
    using R = typename P::R;
    using L = Lat<LAT>;
    constexpr int D = L::D;
    Node nd = node_at(k, tile);
    const long long N = k.N;
    const R *psiA = k.fld.psi[sa.pc];
    // the normal and psi of the tile and its halo staged in LDS (FP32 arithmetic)
    constexpr bool LDS = sizeof(R) == 4;
    using H = Halo1<D, TY>;
    __shared__ R sh[LDS ? D + 1 : 1][LDS ? H::HN : 1];
    if constexpr (LDS) {
        const R *srcs[D + 1];
#pragma unroll
        for (int a = 0; a < D; ++a) srcs[a] = k.fld.nrm + a * N;
        srcs[D] = psiA;
        stage_halo1<LAT, R, D + 1, TY>(k, tile, srcs, sh);
        __syncthreads();
    }
    if (!nd.ok) return;
    const int x = nd.x, y = nd.y, z = nd.z;
    const uint32_t n = node_index(k, nd);
    const R *mac = k.fld.mac[sa.lev];
    const R s = (R)k.fld.sc->scale;
    const Nbhd nb = make_nbhd(k, x, y, z);
    // grad rhoN = -n sqrt(|grad rhoN|^2 + eps_n^2), from the geometry kernel's n and |grad rhoN|
    const R G = ld(k.fld.G[sa.lev], n);
    const R den = sqrt(G * G + k.eps_n * k.eps_n);
    R g[3] = {0, 0, 0}, gp[3] = {0, 0, 0}, nv[3] = {0, 0, 0}, kappa = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        if constexpr (LDS) {
            kappa -= lat_deriv_lds<LAT, TY, R>(nb, sh[a], H::self(), R(1), a, a);
            gp[a] = lat_deriv_lds<LAT, TY, R>(nb, sh[D], H::self(), s, a, -1);
            nv[a] = sh[a][H::self()];
        } else {
            kappa -= lat_deriv<LAT, R>(nb, k.fld.nrm + a * N, n, R(1), a, a);
            gp[a] = lat_deriv<LAT, R>(nb, psiA, n, s, a, -1);
            nv[a] = ld(k.fld.nrm + a * N, n);
        }
        g[a] = -nv[a] * den;
    }
    R psi_st;  // stored (unscaled) psi
    if constexpr (LDS) psi_st = sh[D][H::self()];
    else psi_st = ld(psiA, n);
    const R psi = s * psi_st;
    R Fs[3] = {0, 0, 0};
    // Near saturation the FP32 modes evaluate eq 8 and the Marangoni prefactor of
    // eq 9 in FP64: there 1 - psi/psi_inf is small (1.2e-4 at the CMC of E0 = 0.1)
    // and FP32 rounding of psi s and psi/psi_inf would cost up to 1e-3 of it.
    // Above psi = 0.9 psi_inf, psi = s psi_st, 1 - psi/psi_inf (by log1p), the CMC
    // test and psi_inf - psi are FP64; below it FP32 keeps ~1e-6 relative.
    const bool sat64 = sizeof(R) == 4 && !k.eos_linear && k.E0 != R(0) && psi > R(0.9) * k.psi_inf;
    if (sat64) {
        const double pd = k.fld.sc->scale * (double)psi_st;
        if (pd < k.cmc_d) {
            const R sigma = (R)(k.sigma0_d * (1.0 + k.E0_d * log1p(-pd / k.psi_inf_d)));
            const R mar = (R)(0.5 * (double)G * k.sigma0_d * k.E0_d / (k.psi_inf_d - pd));
            R ndg = 0;
#pragma unroll
            for (int a = 0; a < D; ++a) ndg += nv[a] * gp[a];
#pragma unroll
            for (int a = 0; a < D; ++a) Fs[a] = R(-0.5) * sigma * kappa * g[a] - mar * (gp[a] - ndg * nv[a]);
        } else {
#pragma unroll
            for (int a = 0; a < D; ++a) Fs[a] = R(-0.5) * k.sigma_min * kappa * g[a];
        }
    } else if (k.E0 == R(0)) {
#pragma unroll
        for (int a = 0; a < D; ++a) Fs[a] = R(-0.5) * k.sigma0 * kappa * g[a];
    } else if (k.eos_linear) {
        // Sec 3.2: d sigma / d psi = -sigma0 E0 / psi_inf at every psi
        R sigma = k.sigma0 * (R(1) - k.E0 * psi / k.psi_inf);
        R ndg = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) ndg += nv[a] * gp[a];
        R mar = R(0.5) * G * k.sigma0 * k.E0 / k.psi_inf;
#pragma unroll
        for (int a = 0; a < D; ++a) Fs[a] = R(-0.5) * sigma * kappa * g[a] - mar * (gp[a] - ndg * nv[a]);
    } else if (psi < k.cmc) {
        R sigma = k.sigma0 * (R(1) + k.E0 * log(R(1) - psi / k.psi_inf));
        R ndg = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) ndg += nv[a] * gp[a];
        R mar = R(0.5) * G * k.sigma0 * k.E0 / (k.psi_inf - psi);
#pragma unroll
        for (int a = 0; a < D; ++a) Fs[a] = R(-0.5) * sigma * kappa * g[a] - mar * (gp[a] - ndg * nv[a]);
    } else {
#pragma unroll
        for (int a = 0; a < D; ++a) Fs[a] = R(-0.5) * k.sigma_min * kappa * g[a];
    }
    const R rR = ld(mac, n), rB = ld(mac + N, n);
    const R rho = rR + rB, irho = R(1) / rho;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        R Fa = Fs[a] + (rho - k.rho_ref) * k.grav[a];
        const R ua = (ld(mac + (3 + a) * N, n) + R(0.5) * Fa) * irho;
        st(k.fld.F + a * N, n, Fa);
        st(k.fld.u + a * N, n, ua);
        if (k.qon) st(k.fld.qf + a * N, n, (k.qcoef[0] * rR + k.qcoef[1] * rB) * ua);
    }
}
template <int LAT, class P, int TY> __global__ __launch_bounds__(256) void k_force(KP<typename P::R> k)
{
    force_body<LAT, P, TY>(k, xcd_tile((int)blockIdx.x, (int)gridDim.x), step_args(k));
}
template <int LAT, class P, int TY>
__global__ __launch_bounds__(256) void kb_force(const KP<typename P::R> *tab, const int *prefix, int ninst, StepArgs sa)
{
    int inst, local;
    batch_tile(prefix, ninst, inst, local);
    force_body<LAT, P, TY>(tab[inst], local, sa);
}

// ============================================================== collision

// MRT collision in moment space (eqs 1-4 with the equilibria, corrections and
// relaxation rates of Appendix A), the recolouring descriptor of eqs 11-12,
// and push propagation (eq 13) into the other population buffer.
template <int LAT, class P, bool WM>
__device__ __forceinline__ void collide_body(const KP<typename P::R> &k, int tile, const StepArgs &sa)
{
    using R = typename P::R;
    using S = typename P::S;
    using L = Lat<LAT>;
    constexpr int Q = L::Q, D = L::D;
    Node nd = node_at(k, tile);
    if (!nd.ok) return;
    const int x = nd.x, y = nd.y, z = nd.z;
    const long long N = k.N;
    const uint32_t n = node_index(k, nd);
    const S *fin = (const S *)k.fld.f[sa.fc];
    S *fout = (S *)k.fld.f[1 - sa.fc];
    const R *mac = k.fld.mac[sa.lev];

    const Nbhd nb = make_nbhd(k, x, y, z);
    const R rR = ld(mac, n), rB = ld(mac + N, n);
    // the colour function of eq 6, as the macroscopic kernel forms it from rho^R, rho^B
    const R rr = rR * k.irho0[0], bb = rB * k.irho0[1], rN = (rr - bb) / (rr + bb);
    const R rho = rR + rB, irho = R(1) / rho;
    R u[3] = {0, 0, 0}, F[3] = {0, 0, 0}, nv[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < D; ++d) {
        u[d] = ld(k.fld.u + d * N, n);
        F[d] = ld(k.fld.F + d * N, n);
        nv[d] = ld(k.fld.nrm + d * N, n);
    }
    // moments m = M f of the node
    R m[Q];
    if constexpr (P::DEV) {
        R uj[3] = {0, 0, 0};
#pragma unroll
        for (int d = 0; d < D; ++d) uj[d] = u[d] - R(0.5) * F[d] * irho;
        load_moments<LAT, P>(k, fin, n, rR, rB, uj, m);
    } else {
#pragma unroll
        for (int r = 0; r < Q; ++r) m[r] = 0;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
            const R fj = ldu(fin + j * N, n);
#pragma unroll
            for (int r = 0; r < Q; ++r)
                if (L::M[r][j] != 0) m[r] += R(L::M[r][j]) * fj;
        }
    }
    // relaxation rate of the viscous moments (eq 43 and the mu-s_v relation)
    // 1/mu = (1 + rhoN)/(2 mu^R) + (1 - rhoN)/(2 mu^B); s_v = 1/(mu/p + 1/2) = p/mu / (1 + p/(2 mu))
    const R inv_mu = (R(1) + rN) * k.ihmu[0] + (R(1) - rN) * k.ihmu[1];
    const R pk = rR * k.cs2[0] + rB * k.cs2[1];
    const R pm = pk * inv_mu;
    const R sv = pm / (R(1) + R(0.5) * pm);

    // equilibria summed over colours (eq 37 / eq 40)
    R meq[Q], C[Q];
    meq_sum<LAT, R>(k, rR, rB, u, meq);
#pragma unroll
    for (int r = 0; r < Q; ++r) C[r] = 0;
    const R ux = u[0], uy = u[1], uz = u[2];
    // correction terms C^k with Q_a = qcoef_k d_a(rho^k u_a) (Appendix A); every
    // C row is linear in the colour sum of Q_a, which is the derivative of the
    // field qf_a = sum_k qcoef_k rho^k u_a stored by the force kernel
    if (k.qon) {
        R Qs[3] = {0, 0, 0};
#pragma unroll
        for (int a = 0; a < D; ++a) Qs[a] = lat_deriv<LAT, R>(nb, k.fld.qf + a * N, n, R(1), a, a);
        if constexpr (D == 2) {
            C[1] = R(3) * (Qs[0] + Qs[1]);
            C[7] = Qs[0] - Qs[1];
        } else {
            C[4] = Qs[0] + Qs[1] + Qs[2];
            C[5] = R(2) * Qs[0] - Qs[1] - Qs[2];
            C[6] = Qs[1] - Qs[2];
        }
    }
    // forcing term (eq 4) projected with M. F_i = w_i [3 (e_i - u).F + 9 (e_i.u)(e_i.F)]
    // is a second-order polynomial in e_i times w_i, so its moments are combinations
    // of the lattice tables M w, M w e and M w e e
    R Fm[Q];
    {
        const R uF = ux * F[0] + uy * F[1] + uz * F[2];
        const R F3[3] = {R(3) * F[0], R(3) * F[1], R(3) * F[2]};
        const R uFp[6] = {R(9) * ux * F[0], R(9) * uy * F[1], R(9) * uz * F[2], R(9) * (ux * F[1] + uy * F[0]),
                          R(9) * (ux * F[2] + uz * F[0]), R(9) * (uy * F[2] + uz * F[1])};
#pragma unroll
        for (int r = 0; r < Q; ++r) Fm[r] = wpoly<LAT, R>(r, R(-3) * uF, F3, uFp);
    }
    // post-collision moments m* = m - S (m - meq) + (I - S/2)(C + F_m)  (eqs 1-3)
#pragma unroll
    for (int r = 0; r < Q; ++r) {
        R sr;
        if constexpr (D == 2) {
            sr = r == 1 ? R(1.25) : r == 2 ? R(1.14) : (r == 4 || r == 6) ? R(1.6) : (r >= 7) ? sv : R(0);
        } else {
            sr = (r >= 5 && r <= 9) ? sv : R(1);
        }
        m[r] = m[r] - sr * (m[r] - meq[r]) + (R(1) - R(0.5) * sr) * (C[r] + Fm[r]);
    }
    // recolouring descriptor (eqs 11-12): colour share and c = beta rho^R rho^B / rho g/|g|;
    // the geometry kernel's n = -g / sqrt(|g|^2 + eps_n^2) is parallel to -g, so
    // g/|g| = -n/|n| (n = 0 where g = 0)
    const R a = rR * irho;
    R nn = nv[0] * nv[0];
#pragma unroll
    for (int d = 1; d < D; ++d) nn += nv[d] * nv[d];
    const R cf = nn > R(0) ? -k.beta * (a * rB) / sqrt(nn) : R(0);
    R us[3] = {0, 0, 0};
    if constexpr (P::DEV) {
        // packed descriptor; the reference velocity is used as stored (FP16), so that
        // the decoder's reference equals the encoder's
#pragma unroll
        for (int d = 0; d < D; ++d) us[d] = round_h(u[d] + R(0.5) * F[d] * irho);
        DescDev A;
        A.a = a;
        A.rho = rho;
        A.c01 = pack_h2(cf * nv[0], cf * nv[1]);
        A.c2u0 = D == 3 ? pack_h2(cf * nv[2], us[0]) : pack_h2(us[0], us[1]);
        st((DescDev *)k.fld.desc, n, A);
        if constexpr (D == 3) st(desc_dev_b(k), n, pack_h2(us[1], us[2]));
        // deviation modes store f_dag_i - ref_i with ref_i = rho [a phiR_i + (1 - a) phiB_i
        // + w_i (3 e.u* + 4.5 (e.u*)^2 - 1.5 u*^2)]: subtract the moments of ref from m*
        // (rest part: the colour equilibria at u = 0; motion part: the weighted tables)
        R mr[Q];
        const R zero[3] = {0, 0, 0};
        meq_sum<LAT, R>(k, rho * a, rho - rho * a, zero, mr);
        const R uu = us[0] * us[0] + us[1] * us[1] + us[2] * us[2];
        const R c1[3] = {R(3) * rho * us[0], R(3) * rho * us[1], R(3) * rho * us[2]};
        const R h = R(4.5) * rho;
        const R c2[6] = {h * us[0] * us[0], h * us[1] * us[1], h * us[2] * us[2], R(2) * h * us[0] * us[1],
                         R(2) * h * us[0] * us[2], R(2) * h * us[1] * us[2]};
#pragma unroll
        for (int r = 0; r < Q; ++r) m[r] -= mr[r] + wpoly<LAT, R>(r, R(-1.5) * rho * uu, c1, c2);
    } else {
        st((V4<R> *)k.fld.desc, n, V4<R>{a, cf * nv[0], cf * nv[1], cf * nv[2]});
    }
    // propagation with periodic wrap or half-way bounce-back of f_dag_i = (M^-1 m*)_i
    // (deviation modes: minus ref_i)
    Dither dz(n, P::DEV ? k.fld.sc->tick : 0u, 1u);
    // deviation modes: a reflected population is stored in direction opp(i), and
    // ref_i - ref_opp(i) = 6 rho w_i e_i.u*; refl(i) is that term (zero components
    // of e_i skipped), and refl(opp(i)) = -refl(i)
    auto refl = [&](const int i) -> R {
        R eus = R(0);
        bool first = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (L::E[i][d] == 0) continue;
            eus = first ? R(L::E[i][d]) * us[d] : eus + R(L::E[i][d]) * us[d];
            first = false;
        }
        return R(6 * L::W[i]) * rho * eus;
    };
    auto emit = [&](const int i, R v, R rf) {
        const int ex = L::E[i][0], ey = L::E[i][1], ez = L::E[i][2];
        // the first wall axis the population crosses reflects it, with Ladd's moving-wall
        // term -6 w_i rho (e_i . u_w) (a per-wall table; WM false: no wall moves and the
        // term is zero); every index is a compile-time constant
        const bool bx = ex != 0 && nb_wall_axis(nb, 0, ex);
        const bool by = !bx && ey != 0 && nb_wall_axis(nb, 1, ey);
        const bool bz = !bx && !by && ez != 0 && nb_wall_axis(nb, 2, ez);
        const bool bo = bx || by || bz;
        if constexpr (WM) {
            R wt = R(0);
            if (ex != 0) wt = bx ? k.wterm[ex > 0 ? 1 : 0][i] : wt;
            if (ey != 0) wt = by ? k.wterm[ey > 0 ? 3 : 2][i] : wt;
            if (ez != 0) wt = bz ? k.wterm[ez > 0 ? 5 : 4][i] : wt;
            v -= rho * wt;
        }
        if constexpr (P::DEV) {
            if (i != 0) v += bo ? rf : R(0);
        }
        // one store: base at the lower plane of the pair (i, opp(i)), which are at most
        // two planes apart, so the offset stays below 3 N elements
        const int lo = i < L::OPP[i] ? i : L::OPP[i];
        const uint32_t N32 = (uint32_t)N;
        const uint32_t dst = bo ? (uint32_t)(L::OPP[i] - lo) * N32 + n
                                : (uint32_t)(i - lo) * N32 + n + (uint32_t)nb_delta(nb, ex, ey, ez);
        if constexpr (P::DEV) stu(fout + lo * N, dst, from_real_sr<S>(v, dz.next()));
        else stu(fout + lo * N, dst, (S)v);
    };
    {
        R v = 0;
#pragma unroll
        for (int r = 0; r < Q; ++r)
            if (L::MINV[0][r] != 0.0) v += R(L::MINV[0][r]) * m[r];
        emit(0, v, R(0));
    }
    // opposite pairs: the even rows of M^-1 m* are shared, the odd ones change sign
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        if (L::OPP[i] < i) continue;
        R ev = 0, od = 0;
#pragma unroll
        for (int r = 0; r < Q; ++r) {
            if (L::MINV[i][r] == 0.0) continue;
            if (row_even<LAT>(r)) ev += R(L::MINV[i][r]) * m[r];
            else od += R(L::MINV[i][r]) * m[r];
        }
        const R rf = P::DEV ? refl(i) : R(0);
        emit(i, ev + od, rf);
        emit(L::OPP[i], ev - od, -rf);
    }
}
template <int LAT, class P, bool WM> __global__ __launch_bounds__(256) void k_collide(KP<typename P::R> k)
{
    collide_body<LAT, P, WM>(k, xcd_tile((int)blockIdx.x, (int)gridDim.x), step_args(k));
}
template <int LAT, class P, bool WM>
__global__ __launch_bounds__(256) void kb_collide(const KP<typename P::R> *tab, const int *prefix, int ninst, StepArgs sa)
{
    int inst, local;
    batch_tile(prefix, ninst, inst, local);
    collide_body<LAT, P, WM>(tab[inst], local, sa);
}

// ============================================================== macroscopic fields

// rho^R, rho^B of the streamed populations, rebuilt from the recolouring
// descriptors of the nodes they left (eq 11 summed over arrivals), the colour
// function (eq 6) and the momentum sum f e, into mac of the next level.
template <int LAT, class P, int TY>
__device__ __forceinline__ void macro_body(const KP<typename P::R> &k, int tile, const StepArgs &sa)
{
    using R = typename P::R;
    using S = typename P::S;
    using L = Lat<LAT>;
    constexpr int Q = L::Q, D = L::D;
    Node nd = node_at(k, tile);
    // The descriptors of the tile and its one-node halo (every source an arrival
    // can come from) staged in LDS, so the 19 per-node reads are LDS reads at
    // fixed offsets instead of global gathers: the packed descriptors of the
    // deviation modes, the (a, c) vectors of FP32 and FP64 (16 and 32 bytes).
    // Halo cells beyond a wall are never read (an arrival across a wall comes
    // from the node itself).
    constexpr int HX = BX + 2, HY = TY + 2, HZ = D == 3 ? 3 : 1, HN = HX * HY * HZ;
    constexpr bool TWO = P::DEV && D == 3;
    using TA = std::conditional_t<P::DEV, DescDev, V4<R>>;
    __shared__ TA sA[HN];
    __shared__ uint32_t sB[TWO ? HN : 1];
    {
        const int bx = tile % k.gx, rr = tile / k.gx, gy = gy_of(k, TY);
        const int ox = bx * BX - 1, oy = (rr % gy) * TY - 1, oz = rr / gy - (D == 3 ? 1 : 0);
        const TA *dA = (const TA *)k.fld.desc;
        const uint32_t *dB = desc_dev_b(k);
        // every thread fetches up to HS cells, all loads issued before the LDS stores
        constexpr int HS = (HN + BX * TY - 1) / (BX * TY);
        const int t0 = (int)(threadIdx.x + BX * threadIdx.y);
        TA va[HS];
        uint32_t vb[HS];
        bool have[HS];
#pragma unroll
        for (int it = 0; it < HS; ++it) {
            const int h = t0 + it * BX * TY;
            int g[3] = {ox + h % HX, oy + (h / HX) % HY, oz + h / (HX * HY)};
            const int ext[3] = {k.nx, k.ny, k.nz};
            bool ok = h < HN;
#pragma unroll
            for (int a = 0; a < D; ++a) {
                if (g[a] >= 0 && g[a] < ext[a]) continue;
                if (k.bc[a]) { ok = false; continue; }
                if (g[a] < 0) g[a] += ext[a];
                while (g[a] >= ext[a]) g[a] -= ext[a];
            }
            have[it] = ok;
            if (ok) {
                const uint32_t gi = (uint32_t)g[0] + (uint32_t)k.nx * ((uint32_t)g[1] + (uint32_t)k.ny * (uint32_t)(D == 3 ? g[2] : 0));
                va[it] = ldu(dA, gi);
                if constexpr (TWO) vb[it] = ldu(dB, gi);
            }
        }
#pragma unroll
        for (int it = 0; it < HS; ++it) {
            const int h = t0 + it * BX * TY;
            if (have[it]) {
                sA[h] = va[it];
                if constexpr (TWO) sB[h] = vb[it];
            }
        }
        __syncthreads();
    }
    if (!nd.ok) return;
    const int x = nd.x, y = nd.y, z = nd.z;
    const long long N = k.N;
    const uint32_t n = node_index(k, nd);
    const S *fin = (const S *)k.fld.f[1 - sa.fc];
    const Nbhd nb = make_nbhd(k, x, y, z);
    // halo cell of this node
    const int hself = (int)(threadIdx.x + 1) + HX * ((int)(threadIdx.y + 1) + HY * (D == 3 ? 1 : 0));
    // sums start at their first term (0 + x is not folded in IEEE arithmetic); the
    // flags are compile-time constants once the loops are unrolled
    R rR = 0, rB = 0, j[3] = {0, 0, 0};
    bool jset[3] = {false, false, false}, rset = false;
    R m[P::DEV ? Q : 1];
    bool mset[P::DEV ? Q : 1];
    if constexpr (P::DEV) {
#pragma unroll
        for (int r = 0; r < Q; ++r) { m[r] = 0; mset[r] = false; }
    }
    auto acc = [](R &sum, bool &set, R v) { sum = set ? sum + v : v; set = true; };
    // one arrival: its population (deviation modes: plus the reference of the node it
    // left) and its recoloured share of rho^R, rho^B
    auto arrive = [&](const int q) -> R {
        bool bo;
        R fq = to_real(ldu(fin + q * N, n));
        R as, c[3] = {0, 0, 0};
        if constexpr (P::DEV) {
            // decode with the reference of the node the population left (x - e_q, or
            // the node itself across a wall)
            const int ex = L::E[q][0], ey = L::E[q][1], ez = L::E[q][2];
            bo = nb_wall(nb, -ex, -ey, -ez);
            const int hs = bo ? hself : hself - ex - HX * (ey + HY * ez);
            const DescDev A = sA[hs];
            R us[3] = {0, 0, 0};
            c[0] = h_lo(A.c01);
            c[1] = h_hi(A.c01);
            if constexpr (D == 3) {
                const uint32_t Bv = sB[hs];
                c[2] = h_lo(A.c2u0);
                us[0] = h_hi(A.c2u0);
                us[1] = h_lo(Bv);
                us[2] = h_hi(Bv);
            } else {
                us[0] = h_lo(A.c2u0);
                us[1] = h_hi(A.c2u0);
            }
            as = A.a;
            fq += reference<LAT, R>(k, q, R(1), A.rho, as, us);
        } else {
            const int ex = L::E[q][0], ey = L::E[q][1], ez = L::E[q][2];
            bo = nb_wall(nb, -ex, -ey, -ez);
            const V4<R> A = sA[bo ? hself : hself - ex - HX * (ey + HY * ez)];
            as = A.x;
            c[0] = A.y;
            c[1] = A.z;
            c[2] = A.w;
        }
        const R sgn = bo ? R(-1) : R(1);   // a reflected arrival left its source along -e_q
        R ec = R(0);   // zero components of e_q skipped
        bool first = true;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (L::E[q][d] == 0) continue;
            ec = first ? R(L::E[q][d]) * c[d] : ec + R(L::E[q][d]) * c[d];
            first = false;
        }
        ec *= sgn;
        R wgt = k.recolour_literal ? R(L::W[q]) : as * k.rest[0][q] + (R(1) - as) * k.rest[1][q];
        R r = wgt * ec;
        bool rs = rset;
        acc(rR, rset, as * fq + r);
        acc(rB, rs, (R(1) - as) * fq - r);
        return fq;
    };
    {
        const R f0 = arrive(0);
        if constexpr (P::DEV) {
#pragma unroll
            for (int r2 = 0; r2 < Q; ++r2)
                if (L::M[r2][0] != 0 && !conserved_row<LAT>(r2)) acc(m[r2], mset[r2], R(L::M[r2][0]) * f0);
        }
    }
    // opposite pairs: momentum and the odd moment rows take f_q - f_opp(q), the even
    // rows f_q + f_opp(q)
#pragma unroll
    for (int q = 1; q < Q; ++q) {
        if (L::OPP[q] < q) continue;
        const R fa = arrive(q), fb = arrive(L::OPP[q]);
        const R sp = fa + fb, sm = fa - fb;
#pragma unroll
        for (int d = 0; d < D; ++d)
            if (L::E[q][d] != 0) acc(j[d], jset[d], R(L::E[q][d]) * sm);
        if constexpr (P::DEV) {
#pragma unroll
            for (int r2 = 0; r2 < Q; ++r2)
                if (L::M[r2][q] != 0 && !conserved_row<LAT>(r2))
                    acc(m[r2], mset[r2], R(L::M[r2][q]) * (row_even<LAT>(r2) ? sp : sm));
        }
    }
    R *mac = k.fld.mac[1 - sa.lev];
    R rr = rR * k.irho0[0], bb = rB * k.irho0[1];
    st(mac, n, rR);
    st(mac + N, n, rB);
    st(mac + 2 * N, n, (rr - bb) / (rr + bb));
#pragma unroll
    for (int d = 0; d < D; ++d) st(mac + (3 + d) * N, n, j[d]);
    if constexpr (P::DEV) {
        // in place: the node's own slots, after all of its loads
        R uj[3] = {0, 0, 0};
        const R irho = R(1) / (rR + rB);
#pragma unroll
        for (int d = 0; d < D; ++d) uj[d] = j[d] * irho;
        Dither dz(n, k.fld.sc->tick, 2u);
        store_moments<LAT, P>(k, (S *)k.fld.f[1 - sa.fc], n, rR, rB, uj, m, &dz);
    }
}
template <int LAT, class P, int TY> __global__ __launch_bounds__(256) void k_macro(KP<typename P::R> k)
{
    macro_body<LAT, P, TY>(k, xcd_tile((int)blockIdx.x, (int)gridDim.x), step_args(k));
}
template <int LAT, class P, int TY>
__global__ __launch_bounds__(256) void kb_macro(const KP<typename P::R> *tab, const int *prefix, int ninst, StepArgs sa)
{
    int inst, local;
    batch_tile(prefix, ninst, inst, local);
    macro_body<LAT, P, TY>(tab[inst], local, sa);
}

// ============================================================== finite differences

// WENO3 one-sided differences of eqs 26-27 at the centre of a 5-point line.
// With A = eps + (D+D- at i-1)^2, B = eps + (D+D- at i)^2, C = eps + (D+D- at i+1)^2
// the weights 1/(1 + 2 r^2) are B^2/(B^2 + 2A^2) and B^2/(B^2 + 2C^2); both come
// from one reciprocal of the product of their denominators (all terms >= eps^2).
template <class R> __device__ __forceinline__ void weno_pair(const R *P, R eps, R &Dm, R &Dp)
{
    // P[0..4] = Psi at i-2..i+2
    R d_2 = P[1] - P[0], d_1 = P[2] - P[1], d0 = P[3] - P[2], d1 = P[4] - P[3];
    R dd_1 = P[2] - R(2) * P[1] + P[0], dd0 = P[3] - R(2) * P[2] + P[1], dd1 = P[4] - R(2) * P[3] + P[2];
    const R A = eps + dd_1 * dd_1, B = eps + dd0 * dd0, C = eps + dd1 * dd1;
    const R B2 = B * B, den_m = B2 + R(2) * A * A, den_p = B2 + R(2) * C * C;
    const R inv = fast_rcp(den_m * den_p);
    const R wm = B2 * den_p * inv, wp = B2 * den_m * inv;
    Dm = R(0.5) * ((d_1 + d0) - wm * (d_2 - R(2) * d_1 + d0));
    Dp = R(0.5) * ((d_1 + d0) - wp * (d1 - R(2) * d0 + d_1));
}

template <int LAT, class P> __device__ __forceinline__ void fd_body(const KP<typename P::R> &k, int tile, const StepArgs &sa)
{
    using R = typename P::R;
    using L = Lat<LAT>;
    constexpr int D = L::D;
    Node nd = node_at(k, tile);
    if (!nd.ok) return;
    const int x = nd.x, y = nd.y, z = nd.z;
    const long long N = k.N;
    const uint32_t n = node_index(k, nd);
    const R s = (R)k.fld.sc->scale;
    const R *psiA = k.fld.psi[sa.pc], *phiA = k.fld.phi[sa.pc];
    const R *G0 = k.fld.G[sa.lev];
    const R *rN0 = k.fld.mac[sa.lev] + 2 * N;
    const R *uv = k.fld.u;
    const Nbhd nb = make_nbhd(k, x, y, z);
    R divP = 0, divF = 0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        R Pp[5], Pf[5];
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
            const uint32_t q = o == 0 ? n : n + (uint32_t)nb.d[a][slot_of(o)];
            const R sg = (o != 0 && ((nb.mir >> (a * 4 + slot_of(o))) & 1u)) ? R(-1) : R(1);
            // the lazy scale of the stored psi, phi and the mirror sign ride on u_a
            const R su = sg * (s * ld(uv + a * N, q));
            Pp[o + 2] = (ld(psiA, q) * (ld(G0, q) + k.fd_eps)) * su;
            Pf[o + 2] = (ld(phiA, q) * ((R(1) - ld(rN0, q)) + k.fd_eps)) * su;
        }
        // H+ = u+/|u| and H- = |u-|/|u| are exactly 1 or 0 away from the +-upwind_eps band
        R Dm, Dp, ua = ld(uv + a * N, n);
        const bool band = fabs(ua) <= k.upwind_eps;
        const R hp = band ? R(0.5) : (ua > R(0) ? R(1) : R(0));
        const R hm = band ? R(0.5) : (ua < R(0) ? R(1) : R(0));
        weno_pair(Pp, k.weno_eps, Dm, Dp);
        divP += hp * Dm + hm * Dp;
        weno_pair(Pf, k.weno_eps, Dm, Dp);
        divF += hp * Dm + hm * Dp;
    }
    const R psi = s * ld(psiA, n), phi = s * ld(phiA, n);
    // weights of eqs 20-21 with the background support
    const R Gn = ld(G0, n) + k.fd_eps, Xn = (R(1) - ld(rN0, n)) + k.fd_eps;
    const R jj = k.source_mode == 1 ? k.ra * k.psi_inf * phi : k.ra * phi * (k.psi_inf - psi) - k.rd * psi;
    const R Sn = -divP + Gn * jj, Bn = -divF - Gn * jj;
    const R eS = sa.step == 0 ? Sn : R(1.5) * Sn - R(0.5) * ld(k.fld.Sp, n);
    const R eB = sa.step == 0 ? Bn : R(1.5) * Bn - R(0.5) * ld(k.fld.Bp, n);
    // diffusion operator of eq 28 with half-point weights, as printed (the neighbour sums
    // over the stored psi, phi, scaled once)
    R swP = 0, swcP = 0, swF = 0, swcF = 0;
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int o = -1; o <= 1; o += 2) {
            const uint32_t q = n + (uint32_t)nb.d[a][slot_of(o)];
            R wP = R(0.5) * (Gn + (ld(G0, q) + k.fd_eps));
            R wF = R(0.5) * (Xn + ((R(1) - ld(rN0, q)) + k.fd_eps));
            swcP += wP * ld(psiA, q);
            swP += wP;
            swcF += wF * ld(phiA, q);
            swF += wF;
        }
    const R rhP = Gn * psi + R(0.5) * k.Ds * (s * swcP - swP * psi) + eS;
    const R rhF = Xn * phi + R(0.5) * k.Db * (s * swcF - swF * phi) + eB;
    st(k.fld.Sp, n, Sn);
    st(k.fld.Bp, n, Bn);
    // initial guess of the implicit solve: linear extrapolation from the two
    // previous levels where both exist (the other buffer holds level n-1)
    R psig = psi, phig = phi;
    if (sa.extrap) {
        const R sp = (R)k.fld.sc->scale_prev;
        psig = R(2) * psi - sp * ld(k.fld.psi[1 - sa.pc], n);
        phig = R(2) * phi - sp * ld(k.fld.phi[1 - sa.pc], n);
    }
    // the solve's right-hand sides and initial guesses in its colour-split arrays
    // (the geometry kernel of the new level wrote the node weights there)
    const uint32_t j = split_idx(k, x, y, z);
    st(k.fld.rhs2, j, V2<R>{rhP, rhF});
    st(k.fld.cs2, j, V2<R>{psig, phig});
}
template <int LAT, class P> __global__ __launch_bounds__(256) void k_fd(KP<typename P::R> k)
{
    fd_body<LAT, P>(k, xcd_tile((int)blockIdx.x, (int)gridDim.x), step_args(k));
}
template <int LAT, class P>
__global__ __launch_bounds__(256) void kb_fd(const KP<typename P::R> *tab, const int *prefix, int ninst, StepArgs sa)
{
    int inst, local;
    batch_tile(prefix, ninst, inst, local);
    fd_body<LAT, P>(tab[inst], local, sa);
}

// One colour half of a red-black SOR sweep of both implicit systems
// [W - (Dc/2) L_W] chi = rhs with W = G^{n+1} + eps (psi) and X^{n+1} + eps (phi).
// Persistent grid-stride kernel over the nodes of one colour (x = 2i + parity),
// so every lane updates a node and a sweep that is already converged costs one
// small dispatch. The residual of a row before its update feeds a per-sweep
// maximum (one atomic per block); a sweep whose previous maximum is within
// tolerance returns at once.
template <int LAT, class P>
__device__ __forceinline__ void sor_conv(const KP<typename P::R> &k, int color, int sweep, bool *conv)
{
    using R = typename P::R;
    // Convergence, from maxima over the residual slots (one per lane). With omega = 1
    // and no seam classes the black rows are solved exactly by each black half-sweep,
    // so the red residual before the red update of sweep s is the whole residual after
    // sweep s-1: a black half-sweep is skipped once the red half before it found the
    // system converged, and the red half of the next sweep too. Otherwise the
    // pre-update residuals of every row of the previous sweep are tested.
    conv[0] = conv[1] = false;
    {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int fi = 0; fi < 2; ++fi) {
            const double b = wave_max(bits_to_double(*res_slot(k.fld.sorres, fi, RMAX_IDX, lane)));
            double r = -1.0;
            if (k.sor_exact) {
                // red of sweep s >= 2: test of sweep s-1; black of sweep s >= 1: test of sweep s
                const int sw = color == 0 ? sweep - 1 : sweep;
                if (sw >= 1) r = wave_max(bits_to_double(*res_slot(k.fld.sorres, fi, 2 * sw, lane)));
            } else if (sweep > 0) {
                r = fmax(wave_max(bits_to_double(*res_slot(k.fld.sorres, fi, 2 * (sweep - 1), lane))),
                         wave_max(bits_to_double(*res_slot(k.fld.sorres, fi, 2 * (sweep - 1) + 1, lane))));
            }
            conv[fi] = r >= 0.0 && r <= (double)k.tol * b;
        }
    }
}

// Node (x, y, z) lies on the last plane of an axis that is periodic with an odd
// extent (a seam class of the SOR ordering, below).
template <int D, class R> __device__ __forceinline__ bool on_seam(const KP<R> &k, int x, int y, int z)
{
    return ((k.seam & 1) && x == k.nx - 1) || ((k.seam & 2) && y == k.ny - 1) ||
           (D == 3 && (k.seam & 4) && z == k.nz - 1);
}

// Operands of the implicit systems at this step (colour-split arrays of (psi, phi) pairs).
template <class R> struct SorOps {
    const V2<R> *w;      // node weights W = G^{n+1} + eps (psi) and X^{n+1} + eps (phi)
    V2<R> *chi;          // iterates (initial guess on entry)
    const V2<R> *rhs;
    R hdP, hdF, om;
};
template <class R> __device__ __forceinline__ SorOps<R> sor_ops(const KP<R> &k, const StepArgs &)
{
    SorOps<R> a;
    a.w = k.fld.cw2;
    a.chi = k.fld.cs2;
    a.rhs = k.fld.rhs2;
    a.hdP = R(0.5) * k.Ds;
    a.hdF = R(0.5) * k.Db;
    a.om = k.omega;
    return a;
}

// One SOR update of node (x, y, z) in both implicit systems (a converged system is
// left alone), recording its pre-update residual and |rhs|. Face neighbours in the
// interior lie in the other colour plane at the same row offset; across a periodic
// wrap the neighbour's own parity decides its plane (an odd extent keeps it).
template <int LAT, class P>
__device__ __forceinline__ void sor_node(const KP<typename P::R> &k, const SorOps<typename P::R> &a, int x, int y,
                                         int z, const bool *conv, typename P::R *rloc, typename P::R *bloc)
{
    using R = typename P::R;
    constexpr int D = Lat<LAT>::D, NF = 2 * D;
    const int nx = k.nx, ny = k.ny, nz = k.nz;
    const uint32_t n = split_idx(k, x, y, z);
    const uint32_t hx = k.hx, sz = k.hx * (uint32_t)ny;
    // the same x >> 1 in the other colour plane
    const uint32_t o = ((x + y + z) & 1) ? n - k.hn : n + k.hn;
    uint32_t q[6];
    bool on[6];
    on[0] = x > 0 || !k.bc[0];
    q[0] = x > 0 ? o - (uint32_t)(x >> 1) + (uint32_t)((x - 1) >> 1) : split_idx(k, nx - 1, y, z);
    on[1] = x < nx - 1 || !k.bc[0];
    q[1] = x < nx - 1 ? o - (uint32_t)(x >> 1) + (uint32_t)((x + 1) >> 1) : split_idx(k, 0, y, z);
    on[2] = y > 0 || !k.bc[1];
    q[2] = y > 0 ? o - hx : split_idx(k, x, ny - 1, z);
    on[3] = y < ny - 1 || !k.bc[1];
    q[3] = y < ny - 1 ? o + hx : split_idx(k, x, 0, z);
    if constexpr (D == 3) {
        on[4] = z > 0 || !k.bc[2];
        q[4] = z > 0 ? o - sz : split_idx(k, x, y, nz - 1);
        on[5] = z < nz - 1 || !k.bc[2];
        q[5] = z < nz - 1 ? o + sz : split_idx(k, x, y, 0);
    }
    // diag = W_n + sum_f w_f, off = sum_f w_f chi_f over the faces present (a wall
    // face carries no flux), w_f = (Dc/2) (W_n + W_f)/2, for both systems at once.
    // FP32: each face's pairs are loaded as it is accumulated; FP64 (16-byte pairs):
    // all faces are loaded first (measured faster in each mode; same arithmetic).
    const V2<R> Wn = ld(a.w, n), c0 = ld((const V2<R> *)a.chi, n), rhs = ld(a.rhs, n);
    R dP = Wn.x, oP = 0, dF = Wn.y, oF = 0;
    const auto face = [&](const V2<R> &Wf, const V2<R> &cf) {
        const R wP = a.hdP * (R(0.5) * (Wn.x + Wf.x)), wF = a.hdF * (R(0.5) * (Wn.y + Wf.y));
        dP += wP;
        oP += wP * cf.x;
        dF += wF;
        oF += wF * cf.y;
    };
    if constexpr (sizeof(R) == 8) {
        V2<R> Wf[NF], cf[NF];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            Wf[f] = on[f] ? ld(a.w, q[f]) : V2<R>{R(0), R(0)};
            cf[f] = on[f] ? ld((const V2<R> *)a.chi, q[f]) : V2<R>{R(0), R(0)};
        }
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (on[f]) face(Wf[f], cf[f]);
    } else {
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (on[f]) face(ld(a.w, q[f]), ld((const V2<R> *)a.chi, q[f]));
    }
    // the pre-update residual |rhs - (diag chi - off)| and |rhs| feed the maxima; a
    // converged system keeps its value
    V2<R> v = c0;
    if (!conv[0]) {
        rloc[0] = fmax(rloc[0], fabs(rhs.x - (dP * c0.x - oP)));
        bloc[0] = fmax(bloc[0], fabs(rhs.x));
        v.x = (R(1) - a.om) * c0.x + a.om * (rhs.x + oP) / dP;
    }
    if (!conv[1]) {
        rloc[1] = fmax(rloc[1], fabs(rhs.y - (dF * c0.y - oF)));
        bloc[1] = fmax(bloc[1], fabs(rhs.y));
        v.y = (R(1) - a.om) * c0.y + a.om * (rhs.y + oF) / dF;
    }
    st(a.chi, n, v);
}

// One tile of a colour half-sweep: 256 consecutive entries of the colour's index
// space (i, y, z), i fastest, with x = 2 i + parity. A wavefront spans one row of
// 64 same-colour nodes or, on narrow grids, runs on into the next rows, so no lane
// idles at the end of a row. SEAM: the grid has seam classes (the test costs
// registers, so grids without are served by a variant without it).
template <int LAT, class P, bool SEAM>
__device__ __forceinline__ void sor_tile(const KP<typename P::R> &k, const SorOps<typename P::R> &a, int tile,
                                         int color, const bool *conv, typename P::R *rloc, typename P::R *bloc)
{
    const uint32_t hx = (uint32_t)(k.nx + 1) >> 1;
    const uint32_t L = (uint32_t)tile * 256u + threadIdx.x;
    if (L >= hx * (uint32_t)k.ny * (uint32_t)k.nz) return;
    const uint32_t row = udiv(L, hx, k.inv_hx);
    const uint32_t z = udiv(row, (uint32_t)k.ny, k.inv_ny);
    const int y = (int)(row - z * (uint32_t)k.ny);
    const int x = 2 * (int)(L - row * hx) + ((y + (int)z + color) & 1);
    if (x >= k.nx) return;
    if (SEAM && on_seam<Lat<LAT>::D>(k, x, y, z)) return;   // updated with its seam class
    sor_node<LAT, P>(k, a, x, y, z, conv, rloc, bloc);
}

// Seam classes. On a periodic axis of odd extent the parity colouring wraps onto
// itself: the first and the last plane hold face neighbours of the same parity.
// Nodes on the last plane of such an axis leave the red and black half-sweeps;
// after them they are updated by level (the number of such last planes the node
// lies on), each level in two parity half-sweeps. Face neighbours differ in one
// coordinate, so two nodes of one level and one parity are never neighbours:
// each half-sweep is free of races and the order of all updates is fixed.
// Index space of an instance: for each seam axis a in turn, its last plane, the
// other two axes in increasing order with the lower one fastest.
template <int LAT, class P>
__device__ __forceinline__ void sor_seam_node(const KP<typename P::R> &k, const SorOps<typename P::R> &a, long long t,
                                              int level, int color, const bool *conv, typename P::R *rloc,
                                              typename P::R *bloc)
{
    constexpr int D = Lat<LAT>::D;
    const int ext[3] = {k.nx, k.ny, k.nz};
    int axis = -1;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        if (axis >= 0 || !((k.seam >> a) & 1)) continue;
        const long long plane = k.N / ext[a];
        if (t < plane) axis = a;
        else t -= plane;
    }
    if (axis < 0) return;
    const int b0 = axis == 0 ? 1 : 0, b1 = axis == 2 ? 1 : 2;
    int c[3];
    c[axis] = ext[axis] - 1;
    c[b0] = (int)(t % ext[b0]);
    c[b1] = (int)(t / ext[b0]);
    int lv = 0, lowest = -1;
#pragma unroll
    for (int a = 0; a < D; ++a)
        if (((k.seam >> a) & 1) && c[a] == ext[a] - 1) {
            ++lv;
            if (lowest < 0) lowest = a;
        }
    // a node on several last planes is visited once, from its lowest seam axis
    if (lv != level || lowest != axis || ((c[0] + c[1] + c[2]) & 1) != color) return;
    sor_node<LAT, P>(k, a, c[0], c[1], c[2], conv, rloc, bloc);
}

// Number of tiles of one colour of a half-sweep.
template <class R> __host__ __device__ inline int sor_ntiles(const KP<R> &k)
{
    return sor_tiles_of(k.nx, k.ny, k.nz);
}

// One colour half of a red-black SOR sweep of both implicit systems
// [W - (Dc/2) L_W] chi = rhs with W = G^{n+1} + eps (psi) and X^{n+1} + eps (phi).
// Persistent grid-stride kernel over the nodes of one colour (x = 2i + parity),
// so every lane updates a node and a sweep that is already converged costs one
// small dispatch. The residual of a row before its update feeds a per-sweep
// maximum (one atomic per block); a sweep whose previous maximum is within
// tolerance returns at once.
template <int LAT, class P, bool SEAM>
__global__ __launch_bounds__(256) void k_sor(KP<typename P::R> k, int color, int sweep)
{
    using R = typename P::R;
    bool conv[2];
    sor_conv<LAT, P>(k, color, sweep, conv);
    if (conv[0] && conv[1]) return;
    R rloc[2] = {0, 0}, bloc[2] = {0, 0};
    const int ntiles = sor_ntiles(k);
    const SorOps<R> a = sor_ops(k, step_args(k));
    // the grid is a multiple of 8 or covers every tile once, so raw index mod 8 is the XCD
    for (int raw = blockIdx.x; raw < ntiles; raw += gridDim.x)
        sor_tile<LAT, P, SEAM>(k, a, xcd_tile(raw, ntiles), color, conv, rloc, bloc);
    // block maxima of the pre-update residuals of this colour half-sweep; max |rhs| over
    // the rows of both colours during sweep 0 (no convergence test reads it before sweep 1)
    block_max_to_slots(conv[0] ? R(-1) : rloc[0], conv[1] ? R(-1) : rloc[1], k.fld.sorres, 2 * sweep + color);
    if (sweep == 0) block_max_to_slots(bloc[0], bloc[1], k.fld.sorres, RMAX_IDX);
}

// The same half-sweep for a batch of instances: one workgroup per tile of one instance.
template <int LAT, class P, bool SEAM>
__global__ __launch_bounds__(256) void kb_sor(const KP<typename P::R> *tab, const int *prefix, int ninst, StepArgs sa,
                                             int color, int sweep)
{
    using R = typename P::R;
    int inst, local;
    batch_tile(prefix, ninst, inst, local);
    const KP<R> &k = tab[inst];
    bool conv[2];
    sor_conv<LAT, P>(k, color, sweep, conv);
    if (conv[0] && conv[1]) return;
    R rloc[2] = {0, 0}, bloc[2] = {0, 0};
    sor_tile<LAT, P, SEAM>(k, sor_ops(k, sa), local, color, conv, rloc, bloc);
    block_max_to_slots(conv[0] ? R(-1) : rloc[0], conv[1] ? R(-1) : rloc[1], k.fld.sorres, 2 * sweep + color);
    if (sweep == 0) block_max_to_slots(bloc[0], bloc[1], k.fld.sorres, RMAX_IDX);
}

// Sweeps of a batch past the third usually find most instances converged, and one
// workgroup per tile of every instance then costs a dispatch of every tile. There,
// kb_sor_live first records per instance (one wavefront each) which systems the
// coming half-sweep still updates, and kb_sor_late runs that half-sweep on a narrow
// grid over the live instances only: each workgroup strides over the tiles of each
// live instance and feeds that instance's residual maxima once. The updates of a
// colour half-sweep do not depend on their order and the maxima not on their
// grouping, so every instance gets the result of kb_sor.
template <int LAT, class P>
__global__ __launch_bounds__(64) void kb_sor_live(const KP<typename P::R> *tab, int color, int sweep)
{
    const KP<typename P::R> &k = tab[blockIdx.x];
    bool conv[2];
    sor_conv<LAT, P>(k, color, sweep, conv);
    if (threadIdx.x == 0) k.fld.sc->sor_live = (conv[0] ? 0u : 1u) | (conv[1] ? 0u : 2u);
}
template <int LAT, class P, bool SEAM>
__global__ __launch_bounds__(256) void kb_sor_late(const KP<typename P::R> *tab, const int *prefix, int ninst,
                                                  StepArgs sa, int color, int sweep)
{
    using R = typename P::R;
    __shared__ uint32_t live[64];
    __shared__ unsigned long long lmask;
    for (int c0 = 0; c0 < ninst; c0 += 64) {
        if (threadIdx.x < 64) {
            const uint32_t v = c0 + (int)threadIdx.x < ninst ? tab[c0 + threadIdx.x].fld.sc->sor_live : 0u;
            live[threadIdx.x] = v;
            const unsigned long long m = __ballot(v != 0u);
            if (threadIdx.x == 0) lmask = m;
        }
        __syncthreads();
        unsigned long long m = lmask;
        while (m) {
            const int i = __builtin_ctzll(m);
            m &= m - 1;
            const int inst = c0 + i;
            const int nt = prefix[inst + 1] - prefix[inst];
            if ((int)blockIdx.x >= nt) continue;
            const KP<R> &k = tab[inst];
            const uint32_t v = live[i];
            const bool conv[2] = {(v & 1u) == 0u, (v & 2u) == 0u};
            const SorOps<R> a = sor_ops(k, sa);
            R rloc[2] = {0, 0}, bloc[2] = {0, 0};
            for (int t = blockIdx.x; t < nt; t += gridDim.x) sor_tile<LAT, P, SEAM>(k, a, t, color, conv, rloc, bloc);
            block_max_to_slots(conv[0] ? R(-1) : rloc[0], conv[1] ? R(-1) : rloc[1], k.fld.sorres, 2 * sweep + color);
        }
        __syncthreads();   // live and lmask are rewritten for the next 64 instances
    }
}

// One parity half-sweep of one seam level (one thread per entry of the seam index space).
template <int LAT, class P>
__global__ __launch_bounds__(256) void k_sor_seam(KP<typename P::R> k, int level, int color, int sweep)
{
    using R = typename P::R;
    bool conv[2];
    sor_conv<LAT, P>(k, color, sweep, conv);
    if (conv[0] && conv[1]) return;
    R rloc[2] = {0, 0}, bloc[2] = {0, 0};
    sor_seam_node<LAT, P>(k, sor_ops(k, step_args(k)), (long long)blockIdx.x * 256 + threadIdx.x, level, color, conv,
                          rloc, bloc);
    block_max_to_slots(conv[0] ? R(-1) : rloc[0], conv[1] ? R(-1) : rloc[1], k.fld.sorres, 2 * sweep + color);
    if (sweep == 0) block_max_to_slots(bloc[0], bloc[1], k.fld.sorres, RMAX_IDX);
}

// The same for a batch: instance i owns workgroups prefix[i] .. prefix[i+1]-1.
template <int LAT, class P>
__global__ __launch_bounds__(256) void kb_sor_seam(const KP<typename P::R> *tab, const int *prefix, int ninst,
                                                  StepArgs sa, int level, int color, int sweep)
{
    using R = typename P::R;
    int inst, local;
    batch_tile(prefix, ninst, inst, local);
    const KP<R> &k = tab[inst];
    bool conv[2];
    sor_conv<LAT, P>(k, color, sweep, conv);
    if (conv[0] && conv[1]) return;
    R rloc[2] = {0, 0}, bloc[2] = {0, 0};
    sor_seam_node<LAT, P>(k, sor_ops(k, sa), (long long)local * 256 + threadIdx.x, level, color, conv, rloc, bloc);
    block_max_to_slots(conv[0] ? R(-1) : rloc[0], conv[1] ? R(-1) : rloc[1], k.fld.sorres, 2 * sweep + color);
    if (sweep == 0) block_max_to_slots(bloc[0], bloc[1], k.fld.sorres, RMAX_IDX);
}

// Sweep counts of the last solve; LBFD_ESOR when a system never met its tolerance.
// One wavefront: lane l reads residual slot l. Afterwards it clears the slots of
// every half-sweep and of the |rhs| maxima for the next step.
// One wavefront: the sweep counts and max |rhs| of the last solve, and LBFD_ESOR when a
// system did not converge within the nsw sweeps launched.
template <class R> __device__ __forceinline__ void sor_record(const KP<R> &k, int nsw)
{
    DevScalars *sc = k.fld.sc;
    const int lane = threadIdx.x & 63;
    // residual maxima of the sweeps, four sweeps' slots loaded before any is reduced
    const auto res = [&](int fi, int e) { return e <= 2 * nsw ? bits_to_double(*res_slot(k.fld.sorres, fi, e, lane)) : 0.0; };
    for (int fi = 0; fi < 2; ++fi) {
        const double rm = wave_max(bits_to_double(*res_slot(k.fld.sorres, fi, RMAX_IDX, lane)));
        const double lim = (double)k.tol * rm;
        int K = nsw;
        bool ok = false;
        if (k.sor_exact) {
            // whole residual after s sweeps = red residual at the start of sweep s
            for (int s0 = 1; s0 < nsw && !ok; s0 += 4) {
                double v[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) v[i] = res(fi, 2 * (s0 + i));
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int s = s0 + i;
                    if (ok || s >= nsw) continue;
                    if (wave_max(v[i]) <= lim) { K = s; ok = true; }
                }
            }
        } else {
            for (int s0 = 1; s0 <= nsw && !ok; s0 += 4) {
                double v[4], w[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = res(fi, 2 * (s0 + i - 1));
                    w[i] = res(fi, 2 * (s0 + i - 1) + 1);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int s = s0 + i;
                    if (ok || s > nsw) continue;
                    if (fmax(wave_max(v[i]), wave_max(w[i])) <= lim) { K = s; ok = true; }
                }
            }
        }
        if (lane == 0) {
            sc->rmax[fi] = (unsigned long long)__double_as_longlong(rm);
            sc->sweeps[fi] = K;
            if (!ok && sc->status == 0) sc->status = LBFD_ESOR;
        }
    }
}
// batch: one wavefront per instance
// Clears the residual and |rhs| slots (set-up, before the first step).
template <class R> __global__ void k_sor_clear(KP<R> k, int nsw) { sor_slots_clear(k.fld.sorres, nsw); }


// One FD field from FP64 values: psi and phi given as physical values (stored
// divided by the current scale factor), the AB2 histories as they are.
template <class R> __global__ __launch_bounds__(256) void k_import_fd(KP<R> k, int field, const double *src)
{
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    if (n >= k.N) return;
    const uint32_t i = (uint32_t)n;
    const double sc = k.fld.sc->scale;
    switch (field) {
    case LBFD_FIELD_PSI: st(k.fld.psi[k.pc], i, (R)(src[n] / sc)); break;
    case LBFD_FIELD_PHI: st(k.fld.phi[k.pc], i, (R)(src[n] / sc)); break;
    case LBFD_FIELD_SPREV: st(k.fld.Sp, i, (R)src[n]); break;
    default: st(k.fld.Bp, i, (R)src[n]); break;
    }
}

// ============================================================== surrogate coupling

// Input channels of the surrogate (psi/psi_inf, phi/phi_s, rhoN, u/u_s, zeros up to
// 16) on the grid with a periodic halo of 4 nodes: feat is BF16 [nz+8][ny+8][nx+8][16].
template <int LAT, class P>
__global__ __launch_bounds__(256) void k_sg_features(KP<typename P::R> k, uint16_t *feat, float ipsi, float iphi,
                                                    float iu)
{
    constexpr int D = Lat<LAT>::D;
    const int nx = k.nx, ny = k.ny, nz = k.nz;
    const long long px = nx + 8, py = ny + 8, pz = nz + 8;
    const long long t = (long long)blockIdx.x * 256 + threadIdx.x;
    if (t >= px * py * pz) return;
    const int xp = (int)(t % px), yp = (int)((t / px) % py), zp = (int)(t / (px * py));
    const int x = ((xp - 4) % nx + nx) % nx, y = ((yp - 4) % ny + ny) % ny, z = ((zp - 4) % nz + nz) % nz;
    const long long N = k.N;
    const uint32_t n = (uint32_t)(x + nx * (y + ny * z));
    const double sc = k.fld.sc->scale;
    float c[8];
    c[0] = (float)(sc * (double)ld(k.fld.psi[k.pc], n)) * ipsi;
    c[1] = (float)(sc * (double)ld(k.fld.phi[k.pc], n)) * iphi;
    c[2] = (float)ld(k.fld.mac[k.lev] + 2 * N, n);
#pragma unroll
    for (int a = 0; a < 3; ++a) c[3 + a] = a < D ? (float)ld(k.fld.u + a * N, n) * iu : 0.0f;
    c[6] = c[7] = 0.0f;
    sg::u32x4 lo, zero = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int i = 0; i < 4; ++i) lo[i] = (uint32_t)sg::f2bf(c[2 * i]) | ((uint32_t)sg::f2bf(c[2 * i + 1]) << 16);
    sg::u32x4 *d = (sg::u32x4 *)(feat + t * sg::IN_CH);
    d[0] = lo;
    d[1] = zero;
}

// psi and phi of the current state (physical values), FP32 [N][2].
template <class R> __global__ __launch_bounds__(256) void k_sg_snapshot(KP<R> k, float *snap)
{
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    if (n >= k.N) return;
    const double sc = k.fld.sc->scale;
    snap[2 * n] = (float)(sc * (double)ld(k.fld.psi[k.pc], (uint32_t)n));
    snap[2 * n + 1] = (float)(sc * (double)ld(k.fld.phi[k.pc], (uint32_t)n));
}

// Training tiles: the input crop of tile b from the feature grid (edge T + 8) and the
// targets over its T^3 output nodes: the changes of the conserved densities,
// W (psi now - snap) / dpsi_s and X (phi now - snap) / dphi_s, and the weights
// W = G + fd_eps, X = 1 - rhoN + fd_eps (held over the frozen-flow substeps).
template <class R>
__global__ __launch_bounds__(256) void k_sg_tiles(KP<R> k, const uint16_t *feat, const float *snap, const int *org,
                                                 int T, uint16_t *tin, float *tgt, float idpsi, float idphi)
{
    const int b = blockIdx.y;
    const int ox = org[3 * b], oy = org[3 * b + 1], oz = org[3 * b + 2];
    const long long E = T + 8, nin = E * E * E, nout = (long long)T * T * T;
    const long long px = k.nx + 8, py = k.ny + 8;
    const double sc = k.fld.sc->scale;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < nin; t += (long long)gridDim.x * 256) {
        const long long i = t % E, j = (t / E) % E, l = t / (E * E);
        const long long src = ((oz + l) * py + (oy + j)) * px + (ox + i);
        const sg::u32x4 *s = (const sg::u32x4 *)(feat + src * sg::IN_CH);
        sg::u32x4 *d = (sg::u32x4 *)(tin + ((long long)b * nin + t) * sg::IN_CH);
        d[0] = s[0];
        d[1] = s[1];
    }
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < nout; t += (long long)gridDim.x * 256) {
        const long long i = t % T, j = (t / T) % T, l = t / ((long long)T * T);
        const uint32_t n = (uint32_t)((ox + i) + k.nx * ((oy + j) + (long long)k.ny * (oz + l)));
        const float ps = (float)(sc * (double)ld(k.fld.psi[k.pc], n)), ph = (float)(sc * (double)ld(k.fld.phi[k.pc], n));
        const float W = (float)(ld(k.fld.G[k.lev], n) + k.fd_eps);
        const float X = (float)((R(1) - ld(k.fld.mac[k.lev] + 2 * k.N, n)) + k.fd_eps);
        float *o = tgt + ((long long)b * nout + t) * 4;
        o[0] = W * (ps - snap[2 * (long long)n]) * idpsi;
        o[1] = X * (ph - snap[2 * (long long)n + 1]) * idphi;
        o[2] = W;
        o[3] = X;
    }
}

// Candidate of a surrogate update into the other FD buffers, from the network's
// output o[N][7] on the periodic grid (the conservative form: face fluxes
// weighted by the face weights of their field, the exchange by the interface
// weight): psi + dpsi_s A_psi / W, phi + dphi_s A_phi / X (physical values, as
// an FD update leaves them). Nodes where the result is not finite, or where the
// interface (W >= 1e-3) or the bulk (X >= 1e-3) carries weight and psi or phi
// changes by more than 20 times its change scale (dpsi_s, dphi_s: the 99.9 %
// quantile of the FD update's changes), are counted.
template <class R>
__global__ __launch_bounds__(256) void k_sg_apply(KP<R> k, const float *o, float dpsi, float dphi)
{
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    if (n >= k.N) return;
    const uint32_t i = (uint32_t)n;
    const int x = (int)(n % k.nx), y = (int)((n / k.nx) % k.ny), z = (int)(n / ((long long)k.nx * k.ny));
    const R *G = k.fld.G[k.lev], *rN = k.fld.mac[k.lev] + 2 * k.N;
    const auto Wof = [&](uint32_t m) { return (float)(ld(G, m) + k.fd_eps); };
    const auto Xof = [&](uint32_t m) { return (float)((R(1) - ld(rN, m)) + k.fd_eps); };
    const float ratio = dpsi / dphi;
    const float Wn = Wof(i), Xn = Xof(i);
    float Ap = Wn * o[sg::NOUT * n + 6], Af = -ratio * Wn * o[sg::NOUT * n + 6];
    const int c[3] = {x, y, z}, ext[3] = {k.nx, k.ny, k.nz};
    const long long sd[3] = {1, k.nx, (long long)k.nx * k.ny};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const uint32_t u = (uint32_t)(c[a] + 1 < ext[a] ? n + sd[a] : n - (ext[a] - 1) * sd[a]);
        const uint32_t d = (uint32_t)(c[a] > 0 ? n - sd[a] : n + (ext[a] - 1) * sd[a]);
        Ap -= 0.5f * (Wn + Wof(u)) * o[sg::NOUT * n + a];
        Ap += 0.5f * (Wof(d) + Wn) * o[sg::NOUT * (long long)d + a];
        Af -= 0.5f * (Xn + Xof(u)) * o[sg::NOUT * n + 3 + a];
        Af += 0.5f * (Xof(d) + Xn) * o[sg::NOUT * (long long)d + 3 + a];
    }
    const double sc = k.fld.sc->scale;
    const double dps = (double)dpsi * (double)Ap / (double)Wn, dph = (double)dphi * (double)Af / (double)Xn;
    const double ps = sc * (double)ld(k.fld.psi[k.pc], i) + dps;
    const double ph = sc * (double)ld(k.fld.phi[k.pc], i) + dph;
    st(k.fld.psi[1 - k.pc], i, (R)ps);
    st(k.fld.phi[1 - k.pc], i, (R)ph);
    const bool bad = !(std::isfinite(ps) && std::isfinite(ph)) || (Wn >= 1e-3f && fabs(dps) > 20.0 * (double)dpsi) ||
                     (Xn >= 1e-3f && fabs(dph) > 20.0 * (double)dphi);
    if (bad) atomicAdd(&k.fld.sc->sg_bad, 1u);
}

// Clears the candidate's range counter (one thread).
template <class R> __global__ void k_sg_clear(KP<R> k) { k.fld.sc->sg_bad = 0u; }

// ============================================================== reductions

template <int NV> __device__ __forceinline__ void block_sum_store(double (&v)[NV], double *out)
{
    __shared__ double sh[NV][256];
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[i][t] = v[i];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int i = 0; i < NV; ++i) sh[i][t] += sh[i][t + w];
        __syncthreads();
    }
    if (t == 0)
#pragma unroll
        for (int i = 0; i < NV; ++i) out[i] = sh[i][0];
}

// Per-block FP64 sums of G psi + X phi (the conserved integrand of eqs 20-21)
// at `level`, psi/phi from buffer `buf` times `mult` (mult < 0: the device's
// rescaling factor, which turns stored values into physical ones).
template <int LAT, class P>
__device__ __forceinline__ void total_part_body(const KP<typename P::R> &k, int level, int buf, double mult, int blk,
                                                int nblk, int from_split)
{
    using R = typename P::R;
    const long long N = k.N;
    if (mult < 0.0) mult = k.fld.sc->scale;
    double v[1] = {0.0};
    for (long long n = (long long)blk * blockDim.x + threadIdx.x; n < N; n += (long long)nblk * blockDim.x) {
        const uint32_t i = (uint32_t)n;
        double G = (double)(ld(k.fld.G[level], i) + k.fd_eps);
        double X = (double)((R(1) - ld(k.fld.mac[level] + 2 * N, i)) + k.fd_eps);
        R vp, vf;
        if (from_split) {
            // after the solve: its colour-split iterates become the new level in node order
            const uint32_t yz = udiv(i, (uint32_t)k.nx, k.inv_nx);
            const uint32_t z = udiv(yz, (uint32_t)k.ny, k.inv_ny);
            const uint32_t j = split_idx(k, (int)(i - yz * (uint32_t)k.nx), (int)(yz - z * (uint32_t)k.ny), (int)z);
            const V2<R> c = ld((const V2<R> *)k.fld.cs2, j);
            vp = c.x;
            vf = c.y;
            st(k.fld.psi[buf], i, vp);
            st(k.fld.phi[buf], i, vf);
        } else {
            vp = ld(k.fld.psi[buf], i);
            vf = ld(k.fld.phi[buf], i);
        }
        v[0] += G * (mult * (double)vp) + X * (mult * (double)vf);
    }
    block_sum_store<1>(v, k.fld.part + blk);
}
template <int LAT, class P>
__global__ __launch_bounds__(256) void k_total_part(KP<typename P::R> k, int level, int buf, double mult,
                                                   int from_split)
{
    total_part_body<LAT, P>(k, level, buf, mult, (int)blockIdx.x, (int)gridDim.x, from_split);
}
// batch: instance i owns workgroups prefix[i] .. prefix[i+1]-1
template <int LAT, class P>
__global__ __launch_bounds__(256) void kb_total_part(const KP<typename P::R> *tab, const int *prefix, int ninst,
                                                    int level, int buf, double mult, int from_split)
{
    int inst, local;
    batch_tile(prefix, ninst, inst, local);
    total_part_body<LAT, P>(tab[inst], level, buf, mult, local, prefix[inst + 1] - prefix[inst], from_split);
}
template <class R> __device__ __forceinline__ void total_final_body(const KP<R> &k, long long nblocks, int mode, int nsw)
{
    __shared__ double sh[256];
    const int t = threadIdx.x;
    if (nsw > 0) {
        // after a solve: record its sweeps (first wavefront), then clear its residual
        // slots for the next one (the total's partial sums read none of them)
        if (t < 64) sor_record(k, nsw);
        __syncthreads();
        sor_slots_clear(k.fld.sorres, nsw);
    }
    double a = 0.0;
    for (long long b = t; b < nblocks; b += 256) a += k.fld.part[b];
    sh[t] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) {
        DevScalars *sc = k.fld.sc;
        double M = sh[0];
        if (mode == 0) {
            sc->M0 = M;
            sc->Mlast = M;
            sc->drift_pre = 0.0;
            sc->scale = 1.0;
            sc->scale_prev = 1.0;
        } else if (mode == 2) {
            // probe: the relative change of the total that a candidate makes to the
            // state it starts from (mode 3), at the same weights (nothing else changes)
            sc->drift_pre = sc->Mref != 0.0 ? (M - sc->Mref) / sc->Mref : 0.0;
        } else if (mode == 3) {
            sc->Mref = M;
        } else {
            sc->scale_prev = sc->scale;
            sc->Mlast = M;
            sc->drift_pre = sc->M0 != 0.0 ? (M - sc->M0) / sc->M0 : 0.0;
            sc->scale = (k.rescale && sc->M0 != 0.0 && M != 0.0) ? sc->M0 / M : 1.0;
            if (!isfinite(M) && sc->status == 0) sc->status = LBFD_ENONFINITE;
        }
    }
}
template <class R> __global__ void k_total_final(KP<R> k, long long nblocks, int mode, int nsw)
{
    total_final_body(k, nblocks, mode, nsw);
}
template <class R> __global__ void kb_total_final(const KP<R> *tab, const int *prefix, int mode, int nsw)
{
    const int i = blockIdx.x;
    total_final_body(tab[i], (long long)(prefix[i + 1] - prefix[i]), mode, nsw);
}

// Observables, pass 0: sums and extrema; pass 1: central second moments.
template <int LAT, class P>
__global__ __launch_bounds__(256) void k_obs_part(KP<typename P::R> k, int pass, double cx, double cy, double cz)
{
    using R = typename P::R;
    using L = Lat<LAT>;
    Node nd = node_id(k);
    double v[NRED];
    for (int i = 0; i < NRED; ++i) v[i] = 0.0;
    v[17] = INFINITY;
    v[18] = -INFINITY;
    if (nd.ok) {
        const long long N = k.N, n = lin(k, nd.x, nd.y, nd.z);
        const double s = k.fld.sc->scale;
        const auto *mac = k.fld.mac[k.lev];
        double rR = mac[n], rB = mac[N + n], rN = mac[2 * N + n];
        double w = 0.5 * (1.0 + rN);
        double c[3] = {(double)nd.x, (double)nd.y, (double)nd.z};
        if (pass == 0) {
            double G = k.fld.G[k.lev][n];
            double ps = s * (double)k.fld.psi[k.pc][n], ph = s * (double)k.fld.phi[k.pc][n];
            double Gw = (double)(k.fld.G[k.lev][n] + k.fd_eps);
            double Xw = (double)((R(1) - mac[2 * N + n]) + k.fd_eps);
            v[0] = rR;
            v[1] = rB;
            v[2] = Gw * ps + Xw * ph;
            if (rN >= 0.0) {
                v[3] = 1.0;
                for (int d = 0; d < L::D; ++d) v[4 + d] = k.fld.u[d * N + n];
            }
            v[7] = w;
            for (int d = 0; d < 3; ++d) v[8 + d] = w * c[d];
            v[11] = G;
            v[12] = G * ps;
            double pr = rR * (double)k.cs2[0] + rB * (double)k.cs2[1];
            if (rN > 0.99) { v[13] = pr; v[14] = 1.0; }
            if (rN < -0.99) { v[15] = pr; v[16] = 1.0; }
            if (fabs(rN) <= 0.5) { v[17] = ps; v[18] = ps; }
        } else {
            double d0 = c[0] - cx, d1 = c[1] - cy, d2 = c[2] - cz;
            v[0] = w * d0 * d0; v[1] = w * d1 * d1; v[2] = w * d2 * d2;
            v[3] = w * d0 * d1; v[4] = w * d0 * d2; v[5] = w * d1 * d2;
        }
    }
    // block reduction: sums for 0..16, min for 17, max for 18
    __shared__ double sh[NRED][256];
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
    for (int i = 0; i < NRED; ++i) sh[i][t] = v[i];
    __syncthreads();
    for (int wdt = 128; wdt > 0; wdt >>= 1) {
        if (t < wdt) {
            for (int i = 0; i < 17; ++i) sh[i][t] += sh[i][t + wdt];
            sh[17][t] = fmin(sh[17][t], sh[17][t + wdt]);
            sh[18][t] = fmax(sh[18][t], sh[18][t + wdt]);
        }
        __syncthreads();
    }
    const long long b = blockIdx.x;
    if (t == 0)
        for (int i = 0; i < NRED; ++i) k.fld.part[b * NRED + i] = sh[i][0];
}

__global__ void k_obs_final(const double *part, long long nblocks, double *out)
{
    __shared__ double sh[NRED][256];
    const int t = threadIdx.x;
    double v[NRED];
    for (int i = 0; i < NRED; ++i) v[i] = 0.0;
    v[17] = INFINITY;
    v[18] = -INFINITY;
    for (long long b = t; b < nblocks; b += 256) {
        for (int i = 0; i < 17; ++i) v[i] += part[b * NRED + i];
        v[17] = fmin(v[17], part[b * NRED + 17]);
        v[18] = fmax(v[18], part[b * NRED + 18]);
    }
    for (int i = 0; i < NRED; ++i) sh[i][t] = v[i];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            for (int i = 0; i < 17; ++i) sh[i][t] += sh[i][t + w];
            sh[17][t] = fmin(sh[17][t], sh[17][t + w]);
            sh[18][t] = fmax(sh[18][t], sh[18][t + w]);
        }
        __syncthreads();
    }
    if (t == 0)
        for (int i = 0; i < NRED; ++i) out[i] = sh[i][0];
}

// FP64 export of one field of the current state into a device buffer.
template <int LAT, class P> __global__ __launch_bounds__(256) void k_export(KP<typename P::R> k, int field, double *out)
{
    using R = typename P::R;
    using S = typename P::S;
    using L = Lat<LAT>;
    Node nd = node_id(k);
    if (!nd.ok) return;
    const long long N = k.N, n = lin(k, nd.x, nd.y, nd.z);
    const R *mac = k.fld.mac[k.lev];
    const double s = k.fld.sc->scale;
    switch (field) {
    case LBFD_FIELD_F: {
        const S *f = (const S *)k.fld.f[k.fc];
        if constexpr (P::DEV) {
            R m[L::Q], uj[3] = {0, 0, 0};
            const R rR = mac[n], rB = mac[N + n];
            for (int d = 0; d < L::D; ++d) uj[d] = mac[(3 + d) * N + n] / (rR + rB);
            load_moments<LAT, P>(k, f, n, rR, rB, uj, m);
            for (int i = 0; i < L::Q; ++i) {
                R v = 0;
                for (int r = 0; r < L::Q; ++r) v += R(L::MINV[i][r]) * m[r];
                out[i * N + n] = (double)v;
            }
        } else {
            for (int j = 0; j < L::Q; ++j) out[j * N + n] = (double)to_real(f[j * N + n]);
        }
        break;
    }
    case LBFD_FIELD_RHOR: out[n] = mac[n]; break;
    case LBFD_FIELD_RHOB: out[n] = mac[N + n]; break;
    case LBFD_FIELD_RHON: out[n] = mac[2 * N + n]; break;
    case LBFD_FIELD_U: for (int d = 0; d < L::D; ++d) out[d * N + n] = k.fld.u[d * N + n]; break;
    case LBFD_FIELD_FORCE: for (int d = 0; d < L::D; ++d) out[d * N + n] = k.fld.F[d * N + n]; break;
    case LBFD_FIELD_PSI: out[n] = s * (double)k.fld.psi[k.pc][n]; break;
    case LBFD_FIELD_PHI: out[n] = s * (double)k.fld.phi[k.pc][n]; break;
    case LBFD_FIELD_G: out[n] = k.fld.G[k.lev][n]; break;
    case LBFD_FIELD_SPREV: out[n] = k.fld.Sp[n]; break;
    case LBFD_FIELD_BPREV: out[n] = k.fld.Bp[n]; break;
    default: break;
    }
}

}  // namespace lbfd

// ================================================================== host runtime

using namespace lbfd;

static_assert(sizeof(KP<double>) <= 3072, "kernel parameter block must stay within the kernel-argument limit");

namespace {

enum KernelClass { KC_COLLIDE = 0, KC_MACRO, KC_GEOM, KC_FD, KC_SOR, KC_TOTAL, KC_FORCE, KC_OTHER, KC_COUNT };
const char *kKernelNames[KC_COUNT] = {"collide", "macro", "geom", "fd", "sor", "total", "force", "other"};

struct ProfRec { int kc; hipEvent_t a, b; };

}  // namespace

// Captured two-step graphs. The buffer roles (population, FD and time-level
// selectors) repeat every two steps, so a graph of two steps recorded from one
// role state replays from that state for as long as the handle lives (the
// parameter blocks, buffers and launch budget never change after creation).
// Replay needs steps past the Euler start and an extrapolation history, which
// are the only other per-step inputs of the kernels.
struct StepGraph {
    int fc, pc, lev;
    bool fd_off;
    hipGraphExec_t exec;
};
struct StepGraphs {
    bool on = true;                  // replay when a call advances four or more steps
    hipStream_t cap = nullptr;       // private capture stream (the caller's may be the null stream)
    std::vector<StepGraph> cache;
    // forget the captured graphs (they hold the launch shapes of their capture)
    void drop()
    {
        for (auto &g : cache) hipGraphExecDestroy(g.exec);
        cache.clear();
    }
    void release()
    {
        for (auto &g : cache) hipGraphExecDestroy(g.exec);
        cache.clear();
        if (cap) hipStreamDestroy(cap);
        cap = nullptr;
    }
};

struct lbfd_handle {
    lbfd_params p;
    int Q, D;
    long long N;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    int fc, pc;
    long long step;
    KP<double> kd;
    KP<float> kf;
    dim3 grid, block;
    long long nblocks;
    int tblocks;        // workgroups of the total-surfactant sum
    int sweeps_launch;
    long long fd_hist;  // FD steps since the state was set (extrapolated guess needs one)
    int sor_blocks;     // persistent grid of the SOR sweeps
    int seam_tiles;     // workgroups over the seam index space (0: no seam classes)
    int seam_levels;    // seam levels (periodic axes of odd extent)
    bool prof;
    unsigned prof_mask;  // kernel classes timed when profiling (bit per class)
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    double *obs_out;  // device, NRED doubles (inside the workspace)
    StepGraphs graphs;
    bool fd_off = false;  // LB steps only (psi, phi held): surrogate mode between its updates
    bool kp_dirty = false;  // the parameter block changed after creation (a batch re-uploads its table)
    int dev = 0;          // device current at lbfd_create (the workspace's device)
    // launch shape (a tuning choice; results do not depend on it): rows of 64 x per
    // workgroup of the step's node kernels, the SOR's persistent grid
    int rows = BY;
    int sor_wg_per_cu = 8, sor_narrow = 256, cus = 256;
    dim3 grid4, block4;   // the observables' reduction keeps 64 x 4 workgroups
    long long nblocks4 = 0;
};

// A batch: independent instances (ordinary handles on slices of one workspace)
// advanced together, one launch per kernel class for all of them.
struct lbfd_batch {
    int n;
    std::vector<lbfd_handle *> inst;
    hipStream_t stream;
    void *tab;          // device table of the instances' kernel parameter blocks
    int *prefix_node;   // device: first node tile of each instance (n + 1 entries)
    int *prefix_sor;    // device: first half-sweep tile of each instance (n + 1 entries)
    int *prefix_total;  // device: first total-sum workgroup of each instance (n + 1 entries)
    int *prefix_seam;   // device: first seam workgroup of each instance (n + 1 entries)
    dim3 grid_node, grid_sor, grid_total, grid_seam;
    int seam_levels;    // most seam levels of any instance
    int rows = BY;      // rows of 64 x per workgroup of the node kernels (every instance)
    StepGraphs graphs;
};

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

bool is_dev(int prec) { return prec == LBFD_FP16DEV || prec == LBFD_BF16DEV; }
size_t pop_bytes(int prec) { return prec == LBFD_FP64 ? 8 : prec == LBFD_FP32 ? 4 : 2; }
size_t real_bytes(int prec) { return prec == LBFD_FP64 ? 8 : 4; }

struct Layout {
    size_t f[2], mac[2], desc, G[2], nrm, u, F, qf, sorres, psi[2], phi[2], Sp, Bp, rhs2, cs2, cw2,
        part, sc, obs, total;
};

Layout layout(const lbfd_params *p)
{
    Layout L{};
    const int Q = p->lattice == LBFD_D3Q19 ? 19 : 9, D = p->lattice == LBFD_D3Q19 ? 3 : 2;
    const long long N = (long long)p->nx * p->ny * p->nz;
    const size_t sp = pop_bytes(p->precision), sr = real_bytes(p->precision);
    const int ndesc = is_dev(p->precision) ? 8 : 4;  // one or two packed 4-vectors per node
    const long long nblocks = (long long)((p->nx + BX - 1) / BX) * ((p->ny + BY - 1) / BY) * p->nz;
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t at = o; o += align256(bytes); return at; };
    for (int b = 0; b < 2; ++b) L.f[b] = take(sp * Q * N);
    for (int b = 0; b < 2; ++b) L.mac[b] = take(sr * (3 + D) * N);
    L.desc = take(sr * ndesc * N);
    for (int b = 0; b < 2; ++b) L.G[b] = take(sr * N);
    L.nrm = take(sr * D * N);
    L.u = take(sr * D * N);
    L.F = take(sr * D * N);
    L.qf = take(sr * D * N);
    L.sorres = take(sizeof(unsigned long long) * 2 * (RMAX_IDX + 1) * RSLOTS * RSTRIDE);
    for (int b = 0; b < 2; ++b) L.psi[b] = take(sr * N);
    for (int b = 0; b < 2; ++b) L.phi[b] = take(sr * N);
    L.Sp = take(sr * N);
    L.Bp = take(sr * N);
    // arrays of the implicit solve, two colour planes of ((nx + 1) / 2) ny nz entries each
    const long long NS = 2LL * ((p->nx + 1) / 2) * p->ny * p->nz;
    L.rhs2 = take(2 * sr * NS);
    L.cs2 = take(2 * sr * NS);
    L.cw2 = take(2 * sr * NS);
    const size_t npart = (size_t)NRED * (size_t)nblocks;
    L.part = take(sizeof(double) * (npart > (size_t)TOTAL_BLOCKS ? npart : (size_t)TOTAL_BLOCKS));
    L.sc = take(sizeof(DevScalars));
    L.obs = take(sizeof(double) * NRED);
    L.total = o;
    return L;
}

int check_params(const lbfd_params *p)
{
    if (!p) return LBFD_EINVAL;
    if (p->lattice != LBFD_D2Q9 && p->lattice != LBFD_D3Q19) return LBFD_EINVAL;
    if (p->precision < LBFD_FP64 || p->precision > LBFD_BF16DEV) return LBFD_EINVAL;
    if (p->nx < 4 || p->ny < 4) return LBFD_EINVAL;
    if (p->lattice == LBFD_D2Q9 ? p->nz != 1 : p->nz < 4) return LBFD_EINVAL;
    // 32-bit byte offsets within a plane: N * (largest element, a 4-vector of reals) < 2^32
    if ((long long)p->nx * p->ny * p->nz * (p->precision == LBFD_FP64 ? 32 : 16) >= (1LL << 32)) return LBFD_EINVAL;
    if (!(p->rhoR0 > 0 && p->rhoB0 > 0 && p->muR0 > 0 && p->muB0 > 0)) return LBFD_EINVAL;
    if (!(p->alphaR > 0 && p->alphaR < 1)) return LBFD_EINVAL;
    double alphaB = 1.0 - (p->rhoR0 / p->rhoB0) * (1.0 - p->alphaR);
    if (!(alphaB > 0 && alphaB < 1)) return LBFD_EINVAL;
    if (!(p->psi_inf > 0) || p->E0 < 0 || p->sigma0 < 0) return LBFD_EINVAL;
    if (p->sor_max_sweeps < 1 || p->sor_max_sweeps > MAX_SWEEPS) return LBFD_EINVAL;
    if (!(p->sor_omega > 0 && p->sor_omega < 2)) return LBFD_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (p->bc[a] != LBFD_PERIODIC && p->bc[a] != LBFD_WALL) return LBFD_EINVAL;
    if (p->lattice == LBFD_D2Q9 && p->bc[2] != LBFD_PERIODIC) return LBFD_EINVAL;
    if (p->buoyancy_ref != 0 && p->buoyancy_ref != 1) return LBFD_EINVAL;
    if (p->eos_mode != 0 && p->eos_mode != 1) return LBFD_EINVAL;
    return LBFD_OK;
}

// Rest equilibrium per unit density of a colour with sound-speed parameter al,
// M^-1 m^eq(1, al, 0) written out from eq 37 / eq 40 at u = 0.
template <class Tab> void rest_weights(double al, double cs2, double *out)
{
    double m[QMAX] = {0};
    if (Tab::D == 2) {
        m[0] = 1.0; m[1] = -3.6 * al - 0.4; m[2] = 5.4 * al - 1.4;
    } else {
        m[0] = 1.0; m[4] = 3.0 * cs2;
        for (int r = 16; r < 19; ++r) m[r] = (1.0 - al) / 6.0;
    }
    for (int i = 0; i < Tab::Q; ++i) {
        double a = 0.0;
        for (int r = 0; r < Tab::Q; ++r) a += Tab::MINV[i][r] * m[r];
        out[i] = a;
    }
}

// Axes that are periodic with an odd extent above one (bit a): their last planes
// form the seam classes of the SOR ordering.
int seam_axes(const lbfd_params *p)
{
    const int ext[3] = {p->nx, p->ny, p->nz};
    const int D = p->lattice == LBFD_D3Q19 ? 3 : 2;
    int m = 0;
    for (int a = 0; a < D; ++a)
        if (p->bc[a] == LBFD_PERIODIC && ext[a] > 1 && (ext[a] & 1)) m |= 1 << a;
    return m;
}

// Workgroups of 256 over the seam index space, and the number of seam levels.
void seam_shape(const lbfd_params *p, int *tiles, int *levels)
{
    const int m = seam_axes(p);
    const long long N = (long long)p->nx * p->ny * p->nz;
    const int ext[3] = {p->nx, p->ny, p->nz};
    long long S = 0;
    int lv = 0;
    for (int a = 0; a < 3; ++a)
        if ((m >> a) & 1) {
            S += N / ext[a];
            ++lv;
        }
    *tiles = (int)((S + 255) / 256);
    *levels = lv;
}

template <class R> void fill_kp(KP<R> &k, const lbfd_params *p, char *ws, const Layout &Lo)
{
    const bool three = p->lattice == LBFD_D3Q19;
    k.nx = p->nx; k.ny = p->ny; k.nz = p->nz;
    k.wmove = 0;
    {
        // moving-wall term of the half-way bounce-back per wall and direction: 6 w_i (e_i . u_w)
        const int Q = three ? 19 : 9;
        for (int w = 0; w < 6; ++w)
            for (int i = 0; i < QMAX; ++i) {
                double v = 0.0;
                if (i < Q) {
                    const int *e = three ? D3Q19Tables::E[i] : D2Q9Tables::E[i];
                    const double wi = three ? D3Q19Tables::W[i] : D2Q9Tables::W[i];
                    v = 6.0 * wi * (e[0] * p->wall_u[w][0] + e[1] * p->wall_u[w][1] + e[2] * p->wall_u[w][2]);
                }
                k.wterm[w][i] = (R)v;
                if (k.wterm[w][i] != R(0)) k.wmove = 1;
            }
    }
    k.ihmu[0] = (R)(0.5 / p->muR0);
    k.ihmu[1] = (R)(0.5 / p->muB0);
    k.irho0[0] = (R)(1.0 / p->rhoR0);
    k.irho0[1] = (R)(1.0 / p->rhoB0);
    k.gx = (p->nx + BX - 1) / BX;
    k.gy[0] = p->ny; k.gy[1] = (p->ny + 1) / 2; k.gy[2] = (p->ny + 3) / 4;
    k.N = (long long)p->nx * p->ny * p->nz;
    for (int a = 0; a < 3; ++a) k.bc[a] = p->bc[a];
    for (int w = 0; w < 6; ++w)
        for (int a = 0; a < 3; ++a) k.wall_u[w][a] = (R)p->wall_u[w][a];
    k.rhoR0 = (R)p->rhoR0; k.rhoB0 = (R)p->rhoB0; k.muR0 = (R)p->muR0; k.muB0 = (R)p->muB0;
    // Appendix A: (cs^k)^2 = 0.6 (1 - alpha^k) (2-D), 0.5 (1 - alpha^k) (3-D); eq 42 for alpha^B
    double al[2] = {p->alphaR, 1.0 - (p->rhoR0 / p->rhoB0) * (1.0 - p->alphaR)};
    double cs2[2], qc[2];
    for (int c = 0; c < 2; ++c) {
        cs2[c] = (three ? 0.5 : 0.6) * (1.0 - al[c]);
        qc[c] = three ? (p->q_literal ? 1.0 - cs2[c] : 1.0 - 3.0 * cs2[c]) : 1.8 * al[c] - 0.8;
        k.alpha[c] = (R)al[c];
        k.cs2[c] = (R)cs2[c];
        k.qcoef[c] = (R)qc[c];
    }
    k.qon = (qc[0] != 0.0 || qc[1] != 0.0) ? 1 : 0;
    double rest[2][QMAX] = {{0}};
    for (int c = 0; c < 2; ++c) {
        if (three) rest_weights<D3Q19Tables>(al[c], cs2[c], rest[c]);
        else rest_weights<D2Q9Tables>(al[c], cs2[c], rest[c]);
        for (int i = 0; i < QMAX; ++i) k.rest[c][i] = (R)rest[c][i];
    }
    k.beta = (R)p->beta;
    k.recolour_literal = p->recolour_literal;
    k.sigma0 = (R)p->sigma0; k.E0 = (R)p->E0; k.psi_inf = (R)p->psi_inf;
    k.sigma_min = (R)(p->sigma_min_ratio * p->sigma0);
    k.cmc = (R)(p->E0 > 0 ? p->psi_inf * (1.0 - std::exp(-(1.0 - p->sigma_min_ratio) / p->E0)) : p->psi_inf);
    k.sigma0_d = p->sigma0; k.E0_d = p->E0; k.psi_inf_d = p->psi_inf;
    k.cmc_d = p->E0 > 0 ? p->psi_inf * (1.0 - std::exp(-(1.0 - p->sigma_min_ratio) / p->E0)) : p->psi_inf;
    k.eos_linear = p->eos_mode == 1;
    k.Ds = (R)p->Ds; k.Db = (R)p->Db; k.ra = (R)p->ra; k.rd = (R)p->rd;
    k.source_mode = p->source_mode;
    for (int a = 0; a < 3; ++a) k.grav[a] = (R)p->gravity[a];
    k.rho_ref = (R)p->rhoB0;   // the domain mean replaces it when the fields are set (buoyancy_ref = 1)
    k.omega = (R)p->sor_omega;
    k.tol = (R)p->sor_tol;
    k.seam = seam_axes(p);
    k.inv_hx = 1.0 / (double)((p->nx + 1) / 2);
    k.inv_ny = 1.0 / (double)p->ny;
    k.inv_nx = 1.0 / (double)p->nx;
    k.hx = (uint32_t)((p->nx + 1) / 2);
    k.hn = k.hx * (uint32_t)p->ny * (uint32_t)p->nz;
    k.sor_exact = (p->sor_omega == 1.0 && k.seam == 0) ? 1 : 0;
    k.weno_eps = (R)p->weno_eps;
    k.eps_n = (R)p->eps_n;
    k.fd_eps = (R)p->fd_eps;
    k.upwind_eps = (R)p->upwind_eps;
    k.rescale = p->rescale;
    k.lev = 0; k.fc = 0; k.pc = 0; k.step = 0;
    Fields<R> &F = k.fld;
    for (int b = 0; b < 2; ++b) {
        F.f[b] = ws + Lo.f[b];
        F.mac[b] = (R *)(ws + Lo.mac[b]);
        F.G[b] = (R *)(ws + Lo.G[b]);
        F.psi[b] = (R *)(ws + Lo.psi[b]);
        F.phi[b] = (R *)(ws + Lo.phi[b]);
    }
    F.desc = (void *)(ws + Lo.desc);
    F.nrm = (R *)(ws + Lo.nrm);
    F.u = (R *)(ws + Lo.u);
    F.F = (R *)(ws + Lo.F);
    F.qf = (R *)(ws + Lo.qf);
    F.sorres = (unsigned long long *)(ws + Lo.sorres);
    F.Sp = (R *)(ws + Lo.Sp);
    F.Bp = (R *)(ws + Lo.Bp);
    F.rhs2 = (V2<R> *)(ws + Lo.rhs2);
    F.cs2 = (V2<R> *)(ws + Lo.cs2);
    F.cw2 = (V2<R> *)(ws + Lo.cw2);
    F.part = (double *)(ws + Lo.part);
    F.sc = (DevScalars *)(ws + Lo.sc);
}

hipEvent_t pool_get(lbfd_handle *h)
{
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    hipEventCreate(&e);
    return e;
}

struct Timer {
    lbfd_handle *h;
    int kc;
    hipEvent_t a = nullptr;
    bool on;
    Timer(lbfd_handle *h_, int kc_) : h(h_), kc(kc_), on(h_->prof && ((h_->prof_mask >> kc_) & 1u))
    {
        if (on) {
            a = pool_get(h);
            hipEventRecord(a, h->stream);
        }
    }
    ~Timer()
    {
        if (on) {
            hipEvent_t b = pool_get(h);
            hipEventRecord(b, h->stream);
            h->recs.push_back(ProfRec{kc, a, b});
        }
    }
};

#define LAUNCH(KC, KERNEL, GRID, BLOCK, ...)                                          \
    do {                                                                              \
        Timer _t(h, KC);                                                              \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, h->stream, __VA_ARGS__);           \
    } while (0)

// LAUNCH of a node kernel templated on the rows of its workgroups (the
// handle's tile shape).
#define LAUNCH_TY(ROWS, KC, KERNEL, GRID, BLOCK, ...)                                             \
    do {                                                                                       \
        switch (ROWS) {                                                                        \
        case 1: LAUNCH(KC, (KERNEL<LAT, P, 1>), GRID, BLOCK, __VA_ARGS__); break;               \
        case 2: LAUNCH(KC, (KERNEL<LAT, P, 2>), GRID, BLOCK, __VA_ARGS__); break;               \
        default: LAUNCH(KC, (KERNEL<LAT, P, 4>), GRID, BLOCK, __VA_ARGS__); break;              \
        }                                                                                      \
    } while (0)

// Number of FP64 values lbfd_read_field returns for a field (components x
// nodes), or 0 for an unknown field identifier.
static size_t field_count(const lbfd_handle *h, int field)
{
    switch (field) {
    case LBFD_FIELD_F: return (size_t)h->Q * (size_t)h->N;
    case LBFD_FIELD_U: case LBFD_FIELD_FORCE: return (size_t)h->D * (size_t)h->N;
    case LBFD_FIELD_RHOR: case LBFD_FIELD_RHOB: case LBFD_FIELD_RHON: case LBFD_FIELD_PSI: case LBFD_FIELD_PHI:
    case LBFD_FIELD_G: case LBFD_FIELD_SPREV: case LBFD_FIELD_BPREV: return (size_t)h->N;
    default: return 0;
    }
}

template <int LAT, class P> struct Impl {
    using R = typename P::R;

    static KP<R> &kp(lbfd_handle *h)
    {
        if constexpr (sizeof(R) == 8) return h->kd;
        else return h->kf;
    }

    static void sync_levels(lbfd_handle *h)
    {
        KP<R> &k = kp(h);
        k.lev = (int)(h->step & 1);
        k.fc = h->fc;
        k.pc = h->pc;
        k.step = h->step;
        k.extrap = h->fd_hist >= 1 ? 1 : 0;
        k.nsweeps = h->sweeps_launch;
    }

    // Total of level `level` with psi, phi of buffer `buf` (from_split: take them from
    // the solve's colour-split iterates and store them into `buf` on the way).
    static void totals(lbfd_handle *h, int level, int buf, double mult, int mode, int from_split = 0,
                       int solve_sweeps = 0)
    {
        KP<R> &k = kp(h);
        LAUNCH(KC_TOTAL, (k_total_part<LAT, P>), dim3(h->tblocks), dim3(256), k, level, buf, mult, from_split);
        LAUNCH(KC_TOTAL, (k_total_final<R>), dim3(1), dim3(256), k, (long long)h->tblocks, mode, solve_sweeps);
    }

    static void derived(lbfd_handle *h)
    {
        // geometry and forces of the current level, and (at set-up) the target total
        KP<R> &k = kp(h);
        sync_levels(h);
        LAUNCH(KC_GEOM, (k_geom<LAT, P>), h->grid, h->block, k, k.lev);
        LAUNCH_TY(h->rows, KC_FORCE, k_force, h->grid, h->block, k);
    }

    static int init(lbfd_handle *h, const InitDev &in)
    {
        h->fd_hist = 0;
        h->step = 0;
        h->fc = 0;
        h->pc = 0;
        sync_levels(h);
        KP<R> &k = kp(h);
        LAUNCH(KC_OTHER, (k_init<LAT, P>), h->grid, h->block, k, in);
        LAUNCH(KC_OTHER, (k_sor_clear<R>), dim3(1), dim3(256), k, h->sweeps_launch);
        LAUNCH(KC_GEOM, (k_geom<LAT, P>), h->grid, h->block, k, k.lev);
        clear_scalars(h);
        totals(h, k.lev, k.pc, 1.0, 0);
        if (h->p.buoyancy_ref == 1) {
            // the domain-mean density (exactly conserved) as the buoyancy reference
            lbfd_obs o;
            const int st = observables(h, &o);
            if (st != LBFD_OK && st != LBFD_ENONFINITE && st != LBFD_ESOR) return st;
            set_rho_ref(h, (o.mass_R + o.mass_B) / (double)h->N);
        }
        LAUNCH_TY(h->rows, KC_FORCE, k_force, h->grid, h->block, k);
        return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    // A parameter-block change after creation: captured graphs hold the old block.
    static void set_rho_ref(lbfd_handle *h, double v)
    {
        kp(h).rho_ref = (R)v;
        h->kp_dirty = true;
        if (!h->graphs.cache.empty()) {
            hipStreamSynchronize(h->stream);
            for (auto &g : h->graphs.cache) hipGraphExecDestroy(g.exec);
            h->graphs.cache.clear();
        }
    }

    static void clear_scalars(lbfd_handle *h)
    {
        DevScalars z;
        std::memset(&z, 0, sizeof(z));
        z.scale = 1.0;
        z.scale_prev = 1.0;
        hipMemcpyAsync(kp(h).fld.sc, &z, sizeof(z), hipMemcpyHostToDevice, h->stream);
        hipStreamSynchronize(h->stream);
    }

    static int set_state(lbfd_handle *h, const double *f, const double *rR, const double *rB, const double *psi,
                         const double *phi, const double *Sp, const double *Bp, long long step, double M0)
    {
        const long long N = h->N;
        const size_t nd = (size_t)(h->Q + 6) * N;
        double *d = nullptr;
        if (hipMalloc(&d, nd * sizeof(double)) != hipSuccess) return LBFD_EHIP;
        double *df = d, *drR = d + h->Q * N, *drB = drR + N, *dps = drB + N, *dph = dps + N, *dS = dph + N,
               *dB = dS + N;
        hipMemcpyAsync(df, f, sizeof(double) * h->Q * N, hipMemcpyHostToDevice, h->stream);
        hipMemcpyAsync(drR, rR, sizeof(double) * N, hipMemcpyHostToDevice, h->stream);
        hipMemcpyAsync(drB, rB, sizeof(double) * N, hipMemcpyHostToDevice, h->stream);
        hipMemcpyAsync(dps, psi, sizeof(double) * N, hipMemcpyHostToDevice, h->stream);
        hipMemcpyAsync(dph, phi, sizeof(double) * N, hipMemcpyHostToDevice, h->stream);
        if (Sp) hipMemcpyAsync(dS, Sp, sizeof(double) * N, hipMemcpyHostToDevice, h->stream);
        if (Bp) hipMemcpyAsync(dB, Bp, sizeof(double) * N, hipMemcpyHostToDevice, h->stream);
        h->step = step;
        h->fc = 0;
        h->pc = 0;
        h->fd_hist = 0;
        clear_scalars(h);
        sync_levels(h);
        KP<R> &k = kp(h);
        LAUNCH(KC_OTHER, (k_import<LAT, P>), h->grid, h->block, k, df, drR, drB, dps, dph, Sp ? dS : nullptr,
               Bp ? dB : nullptr);
        LAUNCH(KC_OTHER, (k_sor_clear<R>), dim3(1), dim3(256), k, h->sweeps_launch);
        if (h->p.buoyancy_ref == 1) {
            double m = 0.0;
            for (long long n = 0; n < N; ++n) m += rR[n] + rB[n];
            set_rho_ref(h, m / (double)N);
        }
        derived(h);
        DevScalars z;
        std::memset(&z, 0, sizeof(z));
        z.scale = 1.0;
        z.scale_prev = 1.0;
        z.M0 = M0;
        z.Mlast = M0;
        hipMemcpyAsync(k.fld.sc, &z, sizeof(z), hipMemcpyHostToDevice, h->stream);
        hipError_t e = hipStreamSynchronize(h->stream);
        hipFree(d);
        return e == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    // FD transport of one step (or substep): right-hand sides, the implicit solve
    // by SOR half-sweeps, the sweep count and the total; psi, phi move to the other
    // buffer. The weights of the new level are G[1 - lev] and rhoN of mac[1 - lev].
    static void fd_block(lbfd_handle *h)
    {
        KP<R> &k = kp(h);
        LAUNCH(KC_FD, (k_fd<LAT, P>), h->grid, h->block, k);
        for (int s = 0; s < h->sweeps_launch; ++s) {
            // sweeps past the third usually find both systems converged and return at
            // once: a narrower persistent grid makes that cheaper (the updates of a
            // colour half-sweep do not depend on their order, so the result is the same)
            const dim3 gs(s < 3 ? h->sor_blocks : std::min(h->sor_blocks, h->sor_narrow));
            if (h->seam_levels == 0) {
                LAUNCH(KC_SOR, (k_sor<LAT, P, false>), gs, dim3(256), k, 0, s);
                LAUNCH(KC_SOR, (k_sor<LAT, P, false>), gs, dim3(256), k, 1, s);
                continue;
            }
            LAUNCH(KC_SOR, (k_sor<LAT, P, true>), gs, dim3(256), k, 0, s);
            LAUNCH(KC_SOR, (k_sor<LAT, P, true>), gs, dim3(256), k, 1, s);
            for (int lv = 1; lv <= h->seam_levels; ++lv) {
                LAUNCH(KC_SOR, (k_sor_seam<LAT, P>), dim3(h->seam_tiles), dim3(256), k, lv, 0, s);
                LAUNCH(KC_SOR, (k_sor_seam<LAT, P>), dim3(h->seam_tiles), dim3(256), k, lv, 1, s);
            }
        }
        // the final reduction of the total also records the solve's sweeps and clears its slots
        totals(h, 1 - k.lev, 1 - k.pc, 1.0, 1, 1, h->sweeps_launch);
        h->pc = 1 - h->pc;
        h->fd_hist += 1;
        sync_levels(h);
    }

    // k FD substeps with the flow frozen at the current state: the weights of the
    // new level are set equal to those of the current one (the other level's
    // buffers are free between steps), then k transport updates, then the force
    // from the new psi. The LB populations and the step count do not change.
    static int fd_substeps(lbfd_handle *h, long long ksub)
    {
        if (!h->p.fd_enable || ksub <= 0) return LBFD_OK;
        // the first solve starts from the current value (the other buffer may hold a
        // rejected surrogate candidate rather than the previous level)
        h->fd_hist = 0;
        sync_levels(h);
        KP<R> &k = kp(h);
        const int lev = k.lev;
        const size_t rb = sizeof(R) * (size_t)h->N;
        if (hipMemcpyAsync(k.fld.G[1 - lev], k.fld.G[lev], rb, hipMemcpyDeviceToDevice, h->stream) != hipSuccess ||
            hipMemcpyAsync(k.fld.mac[1 - lev] + 2 * h->N, k.fld.mac[lev] + 2 * h->N, rb, hipMemcpyDeviceToDevice,
                           h->stream) != hipSuccess)
            return LBFD_EHIP;
        for (long long t = 0; t < ksub; ++t) fd_block(h);
        LAUNCH_TY(h->rows, KC_FORCE, k_force, h->grid, h->block, k);
        return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    static int sg_features(lbfd_handle *h, uint16_t *feat, float ipsi, float iphi, float iu)
    {
        sync_levels(h);
        const long long n = (long long)(h->p.nx + 8) * (h->p.ny + 8) * (h->p.nz + 8);
        LAUNCH(KC_OTHER, (k_sg_features<LAT, P>), dim3((unsigned)((n + 255) / 256)), dim3(256), kp(h), feat, ipsi,
               iphi, iu);
        return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    static int sg_snapshot(lbfd_handle *h, float *snap)
    {
        sync_levels(h);
        LAUNCH(KC_OTHER, (k_sg_snapshot<R>), dim3((unsigned)((h->N + 255) / 256)), dim3(256), kp(h), snap);
        return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    static int sg_tiles(lbfd_handle *h, const uint16_t *feat, const float *snap, const int *dorg, int B, int T,
                        uint16_t *tin, float *tgt, float idpsi, float idphi)
    {
        sync_levels(h);
        LAUNCH(KC_OTHER, (k_sg_tiles<R>), dim3(64, (unsigned)B), dim3(256), kp(h), feat, snap, dorg, T, tin, tgt,
               idpsi, idphi);
        return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    // Write the candidate and probe its pre-rescale drift (left in the device scalars).
    static int sg_candidate(lbfd_handle *h, const float *o, float dpsi, float dphi)
    {
        sync_levels(h);
        KP<R> &k = kp(h);
        LAUNCH(KC_OTHER, (k_sg_clear<R>), dim3(1), dim3(1), k);
        totals(h, k.lev, k.pc, -1.0, 3);   // the total the candidate starts from (stored values x scale)
        LAUNCH(KC_OTHER, (k_sg_apply<R>), dim3((unsigned)((h->N + 255) / 256)), dim3(256), k, o, dpsi, dphi);
        totals(h, k.lev, 1 - k.pc, 1.0, 2);
        return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    // Keep the candidate: rescale as an FD update would, swap the buffers, recompute
    // the force; the next solve starts from the old value (no extrapolation history).
    static int sg_accept(lbfd_handle *h)
    {
        sync_levels(h);
        KP<R> &k = kp(h);
        totals(h, k.lev, 1 - k.pc, 1.0, 1);
        h->pc = 1 - h->pc;
        h->fd_hist = 0;
        sync_levels(h);
        LAUNCH_TY(h->rows, KC_FORCE, k_force, h->grid, h->block, k);
        return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    static int read_scalars(lbfd_handle *h, DevScalars *out)
    {
        if (hipMemcpyAsync(out, kp(h).fld.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, h->stream) != hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess)
            return LBFD_EHIP;
        return LBFD_OK;
    }

    static int step_eager(lbfd_handle *h, long long nsteps)
    {
        KP<R> &k = kp(h);
        for (long long t = 0; t < nsteps; ++t) {
            sync_levels(h);
            if (k.wmove) LAUNCH(KC_COLLIDE, (k_collide<LAT, P, true>), h->grid, h->block, k);
            else LAUNCH(KC_COLLIDE, (k_collide<LAT, P, false>), h->grid, h->block, k);
            LAUNCH_TY(h->rows, KC_MACRO, k_macro, h->grid, h->block, k);
            LAUNCH(KC_GEOM, (k_geom<LAT, P>), h->grid, h->block, k, 1 - k.lev);
            if (h->p.fd_enable && !h->fd_off) fd_block(h);
            h->fc = 1 - h->fc;
            h->step += 1;
            sync_levels(h);
            LAUNCH_TY(h->rows, KC_FORCE, k_force, h->grid, h->block, k);
        }
        return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    // One step for every instance of a batch: the same sequence as step(), each
    // kernel class launched once over the tiles of all instances.
    static int batch_eager(lbfd_batch *b, long long nsteps)
    {
        lbfd_handle *h = b->inst[0];   // time levels are common; profiling goes to instance 0
        const KP<R> *tab = (const KP<R> *)b->tab;
        const int n = b->n;
        const dim3 blk(BX, b->rows, 1);
        bool wmove = false;   // some instance has a moving wall
        for (int i = 0; i < n; ++i) wmove = wmove || kp(b->inst[i]).wmove;
        for (long long t = 0; t < nsteps; ++t) {
            StepArgs sa;
            sa.lev = (int)(h->step & 1);
            sa.fc = h->fc;
            sa.pc = h->pc;
            sa.extrap = h->fd_hist >= 1 ? 1 : 0;
            sa.step = h->step;
            if (wmove) LAUNCH(KC_COLLIDE, (kb_collide<LAT, P, true>), b->grid_node, blk, tab, b->prefix_node, n, sa);
            else LAUNCH(KC_COLLIDE, (kb_collide<LAT, P, false>), b->grid_node, blk, tab, b->prefix_node, n, sa);
            LAUNCH_TY(b->rows, KC_MACRO, kb_macro, b->grid_node, blk, tab, b->prefix_node, n, sa);
            LAUNCH(KC_GEOM, (kb_geom<LAT, P>), b->grid_node, blk, tab, b->prefix_node, n, sa, 1 - sa.lev);
            const bool fd = h->p.fd_enable != 0;
            if (fd) {
                LAUNCH(KC_FD, (kb_fd<LAT, P>), b->grid_node, blk, tab, b->prefix_node, n, sa);
                const dim3 g_late((unsigned)std::min((int)b->grid_sor.x, h->sor_narrow));
                for (int s = 0; s < h->sweeps_launch; ++s) {
                    for (int c = 0; c < 2; ++c) {
                        if (s >= 3) {
                            LAUNCH(KC_SOR, (kb_sor_live<LAT, P>), dim3(n), dim3(64), tab, c, s);
                            if (b->seam_levels == 0)
                                LAUNCH(KC_SOR, (kb_sor_late<LAT, P, false>), g_late, dim3(256), tab, b->prefix_sor, n, sa,
                                       c, s);
                            else
                                LAUNCH(KC_SOR, (kb_sor_late<LAT, P, true>), g_late, dim3(256), tab, b->prefix_sor, n, sa,
                                       c, s);
                        } else if (b->seam_levels == 0) {
                            LAUNCH(KC_SOR, (kb_sor<LAT, P, false>), b->grid_sor, dim3(256), tab, b->prefix_sor, n, sa, c, s);
                        } else {
                            LAUNCH(KC_SOR, (kb_sor<LAT, P, true>), b->grid_sor, dim3(256), tab, b->prefix_sor, n, sa, c, s);
                        }
                    }
                    if (b->seam_levels == 0) continue;
                    for (int lv = 1; lv <= b->seam_levels; ++lv) {
                        LAUNCH(KC_SOR, (kb_sor_seam<LAT, P>), b->grid_seam, dim3(256), tab, b->prefix_seam, n, sa, lv,
                               0, s);
                        LAUNCH(KC_SOR, (kb_sor_seam<LAT, P>), b->grid_seam, dim3(256), tab, b->prefix_seam, n, sa, lv,
                               1, s);
                    }
                }
                LAUNCH(KC_TOTAL, (kb_total_part<LAT, P>), b->grid_total, dim3(256), tab, b->prefix_total, n,
                       1 - sa.lev, 1 - sa.pc, 1.0, 1);
                LAUNCH(KC_TOTAL, (kb_total_final<R>), dim3(n), dim3(256), tab, b->prefix_total, 1, h->sweeps_launch);
            }
            for (lbfd_handle *x : b->inst) {
                if (fd) {
                    x->pc = 1 - x->pc;
                    x->fd_hist += 1;
                }
                x->fc = 1 - x->fc;
                x->step += 1;
                sync_levels(x);
            }
            StepArgs sb;
            sb.lev = (int)(h->step & 1);
            sb.fc = h->fc;
            sb.pc = h->pc;
            sb.extrap = h->fd_hist >= 1 ? 1 : 0;
            sb.step = h->step;
            LAUNCH_TY(b->rows, KC_FORCE, kb_force, b->grid_node, blk, tab, b->prefix_node, n, sb);
        }
        return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    // Counters of a handle after two steps (what two eager steps leave behind).
    static void advance_two(lbfd_handle *h)
    {
        if (h->p.fd_enable && !h->fd_off) {
            h->fd_hist += 2;
            // two pc flips leave pc as it was
        }
        h->step += 2;
        sync_levels(h);
    }

    static bool replayable(const lbfd_handle *h)
    {
        return h->step >= 1 && (h->fd_hist >= 1 || !h->p.fd_enable || h->fd_off);
    }

    // Record `two_steps` (which issues two steps on h->stream and advances the
    // counters) on the private stream of `g`, restore the counters and return
    // the instantiated graph, or nullptr when capture is unavailable.
    template <class F>
    static hipGraphExec_t capture(StepGraphs &g, std::vector<lbfd_handle *> &hs, F two_steps)
    {
        if (!g.cap && hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking) != hipSuccess) {
            g.cap = nullptr;
            return nullptr;
        }
        struct Saved { int fc, pc; long long step, fd_hist; hipStream_t stream; };
        std::vector<Saved> sv;
        for (lbfd_handle *x : hs) sv.push_back(Saved{x->fc, x->pc, x->step, x->fd_hist, x->stream});
        for (lbfd_handle *x : hs) x->stream = g.cap;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        bool ok = hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            const int st = two_steps();
            ok = hipStreamEndCapture(g.cap, &graph) == hipSuccess && st == LBFD_OK && graph;
        }
        if (ok) ok = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        if (graph) hipGraphDestroy(graph);
        for (size_t i = 0; i < hs.size(); ++i) {
            lbfd_handle *x = hs[i];
            x->fc = sv[i].fc;
            x->pc = sv[i].pc;
            x->step = sv[i].step;
            x->fd_hist = sv[i].fd_hist;
            x->stream = sv[i].stream;
            sync_levels(x);
        }
        (void)hipGetLastError();
        return ok ? exec : nullptr;
    }

    static hipGraphExec_t graph_for(StepGraphs &g, std::vector<lbfd_handle *> &hs, const std::function<int()> &two)
    {
        const lbfd_handle *h = hs[0];
        const int lev = (int)(h->step & 1);
        for (auto &e : g.cache)
            if (e.fc == h->fc && e.pc == h->pc && e.lev == lev && e.fd_off == h->fd_off) return e.exec;
        hipGraphExec_t ex = capture(g, hs, two);
        if (ex) g.cache.push_back(StepGraph{h->fc, h->pc, lev, h->fd_off, ex});
        return ex;
    }

    // Steps of one handle: eager launches, or replays of a captured two-step
    // graph once the replay conditions hold (results are identical).
    static int step(lbfd_handle *h, long long nsteps)
    {
        if (!h->graphs.on || h->prof || nsteps < 4) return step_eager(h, nsteps);
        while (nsteps > 0 && !replayable(h)) {
            const int st = step_eager(h, 1);
            if (st != LBFD_OK) return st;
            --nsteps;
        }
        std::vector<lbfd_handle *> hs{h};
        hipGraphExec_t ex = nsteps >= 2 ? graph_for(h->graphs, hs, [h]() { return step_eager(h, 2); }) : nullptr;
        if (!ex) return step_eager(h, nsteps);
        for (; nsteps >= 2; nsteps -= 2) {
            if (hipGraphLaunch(ex, h->stream) != hipSuccess) return LBFD_EHIP;
            advance_two(h);
        }
        return nsteps ? step_eager(h, nsteps) : LBFD_OK;
    }

    static int batch_step(lbfd_batch *b, long long nsteps)
    {
        lbfd_handle *h = b->inst[0];
        if (!b->graphs.on || h->prof || nsteps < 4) return batch_eager(b, nsteps);
        while (nsteps > 0 && !replayable(h)) {
            const int st = batch_eager(b, 1);
            if (st != LBFD_OK) return st;
            --nsteps;
        }
        // every instance launches on instance 0's stream, the only one captured
        std::vector<lbfd_handle *> hs(b->inst.begin(), b->inst.end());
        hipGraphExec_t ex = nsteps >= 2 ? graph_for(b->graphs, hs, [b]() { return batch_eager(b, 2); }) : nullptr;
        if (!ex) return batch_eager(b, nsteps);
        for (; nsteps >= 2; nsteps -= 2) {
            if (hipGraphLaunch(ex, h->stream) != hipSuccess) return LBFD_EHIP;
            for (lbfd_handle *x : b->inst) advance_two(x);
        }
        return nsteps ? batch_eager(b, nsteps) : LBFD_OK;
    }

    // Upload the instances' parameter blocks (per-step selectors are passed per launch).
    static int batch_table(lbfd_batch *b)
    {
        std::vector<KP<R>> host(b->n);
        for (int i = 0; i < b->n; ++i) {
            sync_levels(b->inst[i]);
            host[i] = kp(b->inst[i]);
        }
        if (hipMemcpy(b->tab, host.data(), sizeof(KP<R>) * b->n, hipMemcpyHostToDevice) != hipSuccess) return LBFD_EHIP;
        return LBFD_OK;
    }

    static int observables(lbfd_handle *h, lbfd_obs *o)
    {
        KP<R> &k = kp(h);
        sync_levels(h);
        double r0[NRED], r1[NRED];
        LAUNCH(KC_OTHER, (k_obs_part<LAT, P>), h->grid4, h->block4, k, 0, 0.0, 0.0, 0.0);
        LAUNCH(KC_OTHER, k_obs_final, dim3(1), dim3(256), k.fld.part, h->nblocks4, h->obs_out);
        hipMemcpyAsync(r0, h->obs_out, sizeof(r0), hipMemcpyDeviceToHost, h->stream);
        DevScalars sc;
        hipMemcpyAsync(&sc, k.fld.sc, sizeof(sc), hipMemcpyDeviceToHost, h->stream);
        if (hipStreamSynchronize(h->stream) != hipSuccess) return LBFD_EHIP;
        std::memset(o, 0, sizeof(*o));
        o->step = h->step;
        o->mass_R = r0[0];
        o->mass_B = r0[1];
        o->total_surf = r0[2];
        o->nsum = r0[3];
        for (int d = 0; d < 3; ++d) o->velocity[d] = r0[3] > 0 ? r0[4 + d] / r0[3] : 0.0;
        o->wsum = r0[7];
        for (int d = 0; d < 3; ++d) o->centroid[d] = r0[7] > 0 ? r0[8 + d] / r0[7] : 0.0;
        o->psi_av = r0[11] > 0 ? r0[12] / r0[11] : 0.0;
        o->p_in = r0[14] > 0 ? r0[13] / r0[14] : 0.0;
        o->p_out = r0[16] > 0 ? r0[15] / r0[16] : 0.0;
        o->psi_min = r0[17];
        o->psi_max = r0[18];
        LAUNCH(KC_OTHER, (k_obs_part<LAT, P>), h->grid4, h->block4, k, 1, o->centroid[0], o->centroid[1],
               o->centroid[2]);
        LAUNCH(KC_OTHER, k_obs_final, dim3(1), dim3(256), k.fld.part, h->nblocks4, h->obs_out);
        hipMemcpyAsync(r1, h->obs_out, sizeof(r1), hipMemcpyDeviceToHost, h->stream);
        if (hipStreamSynchronize(h->stream) != hipSuccess) return LBFD_EHIP;
        for (int i = 0; i < 6; ++i) o->second[i] = r0[7] > 0 ? r1[i] / r0[7] : 0.0;
        o->drift_pre = sc.drift_pre;
        o->sor_sweeps[0] = sc.sweeps[0];
        o->sor_sweeps[1] = sc.sweeps[1];
        o->status = sc.status;
        o->deformation = deformation(o->second, h->D);
        return sc.status;
    }

    static double deformation(const double *m, int D)
    {
        // eigenvalues of the symmetric 2x2 or 3x3 second-moment tensor; axes ~ sqrt
        double lmax, lmin;
        if (D == 2) {
            double tr = m[0] + m[1], df = m[0] - m[1];
            double r = std::sqrt(0.25 * df * df + m[3] * m[3]);
            lmax = 0.5 * tr + r;
            lmin = 0.5 * tr - r;
        } else {
            double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5];
            double q = (a + b + c) / 3.0;
            double p1 = d * d + e * e + f * f;
            double p2 = (a - q) * (a - q) + (b - q) * (b - q) + (c - q) * (c - q) + 2.0 * p1;
            double pp = std::sqrt(p2 / 6.0);
            if (pp == 0.0) { lmax = lmin = q; }
            else {
                double B[6] = {(a - q) / pp, (b - q) / pp, (c - q) / pp, d / pp, e / pp, f / pp};
                double detB = B[0] * (B[1] * B[2] - B[5] * B[5]) - B[3] * (B[3] * B[2] - B[5] * B[4]) +
                              B[4] * (B[3] * B[5] - B[1] * B[4]);
                double rr = detB / 2.0;
                double phi = rr <= -1 ? M_PI / 3.0 : rr >= 1 ? 0.0 : std::acos(rr) / 3.0;
                lmax = q + 2.0 * pp * std::cos(phi);
                lmin = q + 2.0 * pp * std::cos(phi + 2.0 * M_PI / 3.0);
            }
        }
        double L = std::sqrt(std::fmax(lmax, 0.0)), B = std::sqrt(std::fmax(lmin, 0.0));
        return L + B > 0 ? (L - B) / (L + B) : 0.0;
    }

    // psi, phi (the force is recomputed from the new psi) or the AB2 histories.
    static int write_field(lbfd_handle *h, int field, const double *host, size_t count)
    {
        if (field != LBFD_FIELD_PSI && field != LBFD_FIELD_PHI && field != LBFD_FIELD_SPREV &&
            field != LBFD_FIELD_BPREV)
            return LBFD_EUNSUPPORTED;
        if (!host || count != (size_t)h->N) return LBFD_EINVAL;
        double *d = nullptr;
        if (hipMalloc(&d, count * sizeof(double)) != hipSuccess) return LBFD_EHIP;
        sync_levels(h);
        KP<R> &k = kp(h);
        hipMemcpyAsync(d, host, count * sizeof(double), hipMemcpyHostToDevice, h->stream);
        LAUNCH(KC_OTHER, (k_import_fd<R>), dim3((unsigned)((h->N + 255) / 256)), dim3(256), k, field, d);
        if (field == LBFD_FIELD_PSI) LAUNCH_TY(h->rows, KC_FORCE, k_force, h->grid, h->block, k);
        hipError_t e = hipStreamSynchronize(h->stream);
        hipFree(d);
        return e == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    // FP64 export of one field through the device staging buffer d (count
    // doubles, at least the field's size), then to host memory; synchronous.
    static int export_via(lbfd_handle *h, int field, double *host, size_t count, double *d)
    {
        sync_levels(h);
        LAUNCH(KC_OTHER, (k_export<LAT, P>), h->grid, h->block, kp(h), field, d);
        if (hipMemcpyAsync(host, d, count * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess)
            return LBFD_EHIP;
        return hipStreamSynchronize(h->stream) == hipSuccess ? LBFD_OK : LBFD_EHIP;
    }

    static int read_field(lbfd_handle *h, int field, double *host, size_t count)
    {
        if (field_count(h, field) != count || count == 0 || !host) return LBFD_EINVAL;
        double *d = nullptr;
        if (hipMalloc(&d, count * sizeof(double)) != hipSuccess) return LBFD_EHIP;
        int st = export_via(h, field, host, count, d);
        hipFree(d);
        return st;
    }
};

// Launch shape of a handle: rows of 64 x per workgroup of the step's node kernels,
// and the SOR's persistent grid (workgroups of 256 per compute unit, capped at one
// per tile of a colour; a multiple of 8 keeps the XCD-aware tile order) and the
// grid of sweeps past the third. The results do not depend on it.
void apply_shape(lbfd_handle *h, int rows, int wg_per_cu, int narrow)
{
    const lbfd_params *p = &h->p;
    h->rows = rows;
    h->block = dim3(BX, rows, 1);
    h->nblocks = (long long)((p->nx + BX - 1) / BX) * ((p->ny + rows - 1) / rows) * p->nz;
    h->grid = dim3((unsigned)h->nblocks);
    const long long need = sor_tiles_of(p->nx, p->ny, p->nz);
    const long long cap = (long long)wg_per_cu * h->cus;
    h->sor_wg_per_cu = wg_per_cu;
    h->sor_blocks = (int)(need < cap ? need : cap);
    h->sor_narrow = narrow;
}

struct Dispatch {
    int (*init)(lbfd_handle *, const InitDev &);
    int (*set_state)(lbfd_handle *, const double *, const double *, const double *, const double *, const double *,
                     const double *, const double *, long long, double);
    int (*step)(lbfd_handle *, long long);
    int (*observables)(lbfd_handle *, lbfd_obs *);
    int (*read_field)(lbfd_handle *, int, double *, size_t);
    int (*write_field)(lbfd_handle *, int, const double *, size_t);
    int (*batch_step)(lbfd_batch *, long long);
    int (*batch_table)(lbfd_batch *);
    size_t kp_bytes;
    int (*fd_substeps)(lbfd_handle *, long long);
    int (*sg_features)(lbfd_handle *, uint16_t *, float, float, float);
    int (*sg_snapshot)(lbfd_handle *, float *);
    int (*sg_tiles)(lbfd_handle *, const uint16_t *, const float *, const int *, int, int, uint16_t *, float *, float,
                    float);
    int (*sg_candidate)(lbfd_handle *, const float *, float, float);
    int (*sg_accept)(lbfd_handle *);
    int (*read_scalars)(lbfd_handle *, DevScalars *);
    int (*export_via)(lbfd_handle *, int, double *, size_t, double *);
};

template <int LAT, class P> Dispatch make_dispatch()
{
    using I = Impl<LAT, P>;
    return Dispatch{&I::init,        &I::set_state,   &I::step,        &I::observables, &I::read_field,
                    &I::write_field, &I::batch_step,  &I::batch_table, sizeof(KP<typename P::R>),
                    &I::fd_substeps, &I::sg_features, &I::sg_snapshot, &I::sg_tiles,      &I::sg_candidate,
                    &I::sg_accept,   &I::read_scalars, &I::export_via};
}

Dispatch dispatch_for(int lat, int prec)
{
    if (lat == LBFD_D2Q9) {
        switch (prec) {
        case LBFD_FP64: return make_dispatch<0, PrecF64>();
        case LBFD_FP32: return make_dispatch<0, PrecF32>();
        case LBFD_FP16DEV: return make_dispatch<0, PrecF16>();
        default: return make_dispatch<0, PrecB16>();
        }
    }
    switch (prec) {
    case LBFD_FP64: return make_dispatch<1, PrecF64>();
    case LBFD_FP32: return make_dispatch<1, PrecF32>();
    case LBFD_FP16DEV: return make_dispatch<1, PrecF16>();
    default: return make_dispatch<1, PrecB16>();
    }
}

// ---- fixed staging buffer of lbfd_read_field_noalloc ------------------------
// Callers that cannot allocate device memory (code under graph capture, tight
// serving loops) read fields through this file-scope array instead of a
// per-call allocation. Every device the library runs on holds one copy, at its
// own address, until the process ends. Host code never passes the array's name
// to a kernel or a copy (on the host it is only a stand-in symbol): it uses the
// device address hipGetSymbolAddress returns for the current device, looked up
// once per device and kept in scratch_ptr.
constexpr size_t SCRATCH_DOUBLES = (size_t)8 << 20;  // 64 MiB: one scalar field of up to 8 Mi nodes
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Device address of `scratch` on device dev (made current for the lookup, then
// the caller's current device is restored).
int scratch_address(int dev, double **out)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return LBFD_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return LBFD_EHIP;
        if (cur != dev && hipSetDevice(dev) != hipSuccess) return LBFD_EHIP;
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != dev) hipSetDevice(cur);
        if (e != hipSuccess || !ptr) return LBFD_EHIP;
        scratch_ptr[dev] = (double *)ptr;
    }
    *out = scratch_ptr[dev];
    return LBFD_OK;
}

int sticky_status(lbfd_handle *h)
{
    DevScalars sc;
    const DevScalars *d = h->p.precision == LBFD_FP64 ? h->kd.fld.sc : h->kf.fld.sc;
    if (hipMemcpyAsync(&sc, d, sizeof(sc), hipMemcpyDeviceToHost, h->stream) != hipSuccess) return LBFD_EHIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LBFD_EHIP;
    return sc.status;
}

}  // namespace

extern "C" {

int lbfd_workspace_bytes(const lbfd_params *p, size_t *bytes)
{
    int st = check_params(p);
    if (st != LBFD_OK) return st;
    if (!bytes) return LBFD_EINVAL;
    *bytes = layout(p).total;
    return LBFD_OK;
}

int lbfd_create(const lbfd_params *p, void *d_workspace, size_t bytes, void *stream, lbfd_handle **out)
{
    if (!out) return LBFD_EINVAL;
    *out = nullptr;
    int st = check_params(p);
    if (st != LBFD_OK) return st;
    Layout Lo = layout(p);
    if (!d_workspace || bytes < Lo.total) return LBFD_EWORKSPACE;
    if (((uintptr_t)d_workspace & 255) != 0) return LBFD_EWORKSPACE;
    lbfd_handle *h = new (std::nothrow) lbfd_handle();
    if (!h) return LBFD_ENOMEM;
    h->p = *p;
    h->Q = p->lattice == LBFD_D3Q19 ? 19 : 9;
    h->D = p->lattice == LBFD_D3Q19 ? 3 : 2;
    h->N = (long long)p->nx * p->ny * p->nz;
    h->stream = (hipStream_t)stream;
    h->ws = (char *)d_workspace;
    h->ws_bytes = bytes;
    h->fc = h->pc = 0;
    h->step = 0;
    h->block4 = dim3(BX, BY, 1);
    h->nblocks4 = (long long)((p->nx + BX - 1) / BX) * ((p->ny + BY - 1) / BY) * p->nz;
    h->grid4 = dim3((unsigned)h->nblocks4);
    h->tblocks = total_blocks(h->N);
    seam_shape(p, &h->seam_tiles, &h->seam_levels);
    h->sweeps_launch = p->sor_max_sweeps;
    {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipDeviceProp_t prop;
            if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
                h->cus = prop.multiProcessorCount;
        }
    }
    apply_shape(h, BY, 8, 256);
    h->prof = false;
    h->prof_mask = 0xffffffffu;
    if (hipGetDevice(&h->dev) != hipSuccess) h->dev = 0;
    fill_kp(h->kd, p, h->ws, Lo);
    fill_kp(h->kf, p, h->ws, Lo);
    h->obs_out = (double *)(h->ws + Lo.obs);
    *out = h;
    return LBFD_OK;
}

int lbfd_init_fields(lbfd_handle *h, const lbfd_init *in)
{
    if (!h || !in || in->n < 0 || in->n > 16 || !(in->width > 0)) return LBFD_EINVAL;
    InitDev d;
    d.n = in->n;
    for (int i = 0; i < 16; ++i) { d.cx[i] = in->cx[i]; d.cy[i] = in->cy[i]; d.cz[i] = in->cz[i]; d.r[i] = in->r[i]; }
    d.width = in->width;
    d.psi0 = in->psi0;
    d.phi0_out = in->phi0_out;
    d.phi0_in = in->phi0_in;
    d.shear_rate = in->shear_rate;
    if (!(in->psi0 >= 0 && in->psi0 < h->p.psi_inf)) return LBFD_EINVAL;
    return dispatch_for(h->p.lattice, h->p.precision).init(h, d);
}

int lbfd_set_state(lbfd_handle *h, const double *f, const double *rhoR, const double *rhoB, const double *psi,
                   const double *phi, const double *Sprev, const double *Bprev, int64_t step, double M0)
{
    if (!h || !f || !rhoR || !rhoB || !psi || !phi || step < 0) return LBFD_EINVAL;
    return dispatch_for(h->p.lattice, h->p.precision).set_state(h, f, rhoR, rhoB, psi, phi, Sprev, Bprev, step, M0);
}

int lbfd_step(lbfd_handle *h, int64_t n)
{
    if (!h || n < 0) return LBFD_EINVAL;
    return dispatch_for(h->p.lattice, h->p.precision).step(h, n);
}

int lbfd_observables(lbfd_handle *h, lbfd_obs *out)
{
    if (!h || !out) return LBFD_EINVAL;
    return dispatch_for(h->p.lattice, h->p.precision).observables(h, out);
}

int lbfd_read_field(lbfd_handle *h, int32_t field, double *host, size_t count)
{
    if (!h) return LBFD_EINVAL;
    int st = dispatch_for(h->p.lattice, h->p.precision).read_field(h, field, host, count);
    if (st != LBFD_OK) return st;
    return sticky_status(h);
}

int lbfd_read_field_noalloc(lbfd_handle *h, int32_t field, double *host, size_t count)
{
    if (!h || !host) return LBFD_EINVAL;
    const size_t need = field_count(h, field);
    if (need == 0 || count != need) return LBFD_EINVAL;
    if (count > SCRATCH_DOUBLES) return LBFD_ESCRATCH;
    double *d = nullptr;
    int st = scratch_address(h->dev, &d);
    if (st != LBFD_OK) return st;
    st = dispatch_for(h->p.lattice, h->p.precision).export_via(h, field, host, count, d);
    if (st != LBFD_OK) return st;
    return sticky_status(h);
}

int lbfd_set_fd(lbfd_handle *h, int32_t enable)
{
    if (!h) return LBFD_EINVAL;
    h->fd_off = enable == 0;
    return LBFD_OK;
}

int lbfd_set_graphs(lbfd_handle *h, int32_t enable)
{
    if (!h) return LBFD_EINVAL;
    h->graphs.on = enable != 0;
    return LBFD_OK;
}

static int tuning_valid(const lbfd_tuning *t)
{
    return t && (t->rows == 1 || t->rows == 2 || t->rows == 4) && t->sor_wg_per_cu >= 1 && t->sor_wg_per_cu <= 32 &&
           t->sor_narrow >= 8 && t->sor_narrow <= 65536 && t->sor_narrow % 8 == 0;
}

int lbfd_set_tuning(lbfd_handle *h, const lbfd_tuning *t)
{
    if (!h || !tuning_valid(t)) return LBFD_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LBFD_EHIP;
    h->graphs.drop();
    apply_shape(h, t->rows, t->sor_wg_per_cu, t->sor_narrow);
    return LBFD_OK;
}

int lbfd_get_tuning(const lbfd_handle *h, lbfd_tuning *t)
{
    if (!h || !t) return LBFD_EINVAL;
    t->rows = h->rows;
    t->sor_wg_per_cu = h->sor_wg_per_cu;
    t->sor_narrow = h->sor_narrow;
    return LBFD_OK;
}

int lbfd_batch_set_tuning(lbfd_batch *b, const lbfd_tuning *t)
{
    if (!b || !tuning_valid(t)) return LBFD_EINVAL;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return LBFD_EHIP;
    b->graphs.drop();
    std::vector<int> pn(b->n + 1);
    pn[0] = 0;
    for (int i = 0; i < b->n; ++i) {
        lbfd_handle *h = b->inst[i];
        h->graphs.drop();
        apply_shape(h, t->rows, t->sor_wg_per_cu, t->sor_narrow);
        pn[i + 1] = pn[i] + (int)h->nblocks;
    }
    if (hipMemcpy(b->prefix_node, pn.data(), sizeof(int) * (b->n + 1), hipMemcpyHostToDevice) != hipSuccess)
        return LBFD_EHIP;
    b->grid_node = dim3((unsigned)pn[b->n]);
    b->rows = t->rows;
    return LBFD_OK;
}

int lbfd_batch_set_graphs(lbfd_batch *b, int32_t enable)
{
    if (!b) return LBFD_EINVAL;
    b->graphs.on = enable != 0;
    return LBFD_OK;
}

int lbfd_profile(lbfd_handle *h, int32_t enable)
{
    if (!h) return LBFD_EINVAL;
    hipStreamSynchronize(h->stream);
    for (auto &r : h->recs) { h->pool.push_back(r.a); h->pool.push_back(r.b); }
    h->recs.clear();
    h->prof = enable != 0;
    // enable = 1: every kernel class; enable = 1 + (1 << (k + 1)) ...: only the classes set in bits 1..
    unsigned m = (unsigned)enable >> 1;
    h->prof_mask = m ? m : 0xffffffffu;
    return LBFD_OK;
}

int lbfd_profile_read(lbfd_handle *h, int32_t max_kernels, const char **names, double *ms, int64_t *launches,
                      int32_t *n_kernels)
{
    if (!h || !n_kernels) return LBFD_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return LBFD_EHIP;
    double acc[KC_COUNT] = {0};
    int64_t cnt[KC_COUNT] = {0};
    for (auto &r : h->recs) {
        float t = 0.f;
        hipEventElapsedTime(&t, r.a, r.b);
        acc[r.kc] += t;
        cnt[r.kc] += 1;
    }
    int nk = KC_COUNT < max_kernels ? KC_COUNT : max_kernels;
    for (int i = 0; i < nk; ++i) {
        if (names) names[i] = kKernelNames[i];
        if (ms) ms[i] = acc[i];
        if (launches) launches[i] = cnt[i];
    }
    *n_kernels = nk;
    return LBFD_OK;
}

void lbfd_destroy(lbfd_handle *h)
{
    if (!h) return;
    hipStreamSynchronize(h->stream);
    h->graphs.release();
    for (auto &r : h->recs) { hipEventDestroy(r.a); hipEventDestroy(r.b); }
    for (auto e : h->pool) hipEventDestroy(e);
    delete h;
}

// ------------------------------------------------------------------ batches

static int batch_layout(const lbfd_params *p, int32_t n, std::vector<size_t> *offs, size_t *tab_off, size_t *pre_off,
                        size_t *total)
{
    if (!p || n < 1 || n > 65536) return LBFD_EINVAL;
    size_t o = 0;
    long long node_tiles = 0, sor_tiles = 0;
    for (int i = 0; i < n; ++i) {
        int st = check_params(&p[i]);
        if (st != LBFD_OK) return st;
        if (p[i].lattice != p[0].lattice || p[i].precision != p[0].precision || p[i].fd_enable != p[0].fd_enable ||
            p[i].sor_max_sweeps != p[0].sor_max_sweeps)
            return LBFD_EINVAL;
        if (offs) offs->push_back(o);
        o += align256(layout(&p[i]).total);
        node_tiles += (long long)((p[i].nx + BX - 1) / BX) * ((p[i].ny + BY - 1) / BY) * p[i].nz;
        sor_tiles += sor_tiles_of(p[i].nx, p[i].ny, p[i].nz);
    }
    // one launch covers the tiles of all instances: 256 lanes per tile, 32-bit lane ids
    if (node_tiles * 256 > (long long)UINT32_MAX || sor_tiles * 256 > (long long)UINT32_MAX) return LBFD_EINVAL;
    const size_t kpb = dispatch_for(p[0].lattice, p[0].precision).kp_bytes;
    *tab_off = o;
    o += align256(kpb * (size_t)n);
    *pre_off = o;
    o += align256(sizeof(int) * 4 * ((size_t)n + 1));
    *total = o;
    return LBFD_OK;
}

int lbfd_batch_workspace_bytes(const lbfd_params *p, int32_t n, size_t *bytes)
{
    if (!bytes) return LBFD_EINVAL;
    size_t t, pr, tot;
    int st = batch_layout(p, n, nullptr, &t, &pr, &tot);
    if (st != LBFD_OK) return st;
    *bytes = tot;
    return LBFD_OK;
}

void lbfd_batch_destroy(lbfd_batch *b)
{
    if (!b) return;
    if (!b->inst.empty()) hipStreamSynchronize(b->inst[0]->stream);
    b->graphs.release();
    for (lbfd_handle *h : b->inst) lbfd_destroy(h);
    delete b;
}

int lbfd_batch_create(const lbfd_params *p, int32_t n, void *d_workspace, size_t bytes, void *stream, lbfd_batch **out)
{
    if (!out) return LBFD_EINVAL;
    *out = nullptr;
    std::vector<size_t> offs;
    size_t tab_off, pre_off, total;
    int st = batch_layout(p, n, &offs, &tab_off, &pre_off, &total);
    if (st != LBFD_OK) return st;
    if (!d_workspace || bytes < total || ((uintptr_t)d_workspace & 255) != 0) return LBFD_EWORKSPACE;
    lbfd_batch *b = new (std::nothrow) lbfd_batch();
    if (!b) return LBFD_ENOMEM;
    b->n = n;
    b->stream = (hipStream_t)stream;
    char *ws = (char *)d_workspace;
    std::vector<int> pn(n + 1), ps(n + 1), pt(n + 1), pm(n + 1);
    pn[0] = ps[0] = pt[0] = pm[0] = 0;
    b->seam_levels = 0;
    for (int i = 0; i < n; ++i) {
        lbfd_handle *h = nullptr;
        st = lbfd_create(&p[i], ws + offs[i], layout(&p[i]).total, stream, &h);
        if (st != LBFD_OK) {
            lbfd_batch_destroy(b);
            return st;
        }
        b->inst.push_back(h);
        pn[i + 1] = pn[i] + (int)h->nblocks;
        ps[i + 1] = ps[i] + sor_tiles_of(p[i].nx, p[i].ny, p[i].nz);
        pt[i + 1] = pt[i] + h->tblocks;
        pm[i + 1] = pm[i] + h->seam_tiles;
        if (h->seam_levels > b->seam_levels) b->seam_levels = h->seam_levels;
    }
    b->tab = ws + tab_off;
    b->prefix_node = (int *)(ws + pre_off);
    b->prefix_sor = b->prefix_node + (n + 1);
    b->prefix_total = b->prefix_sor + (n + 1);
    b->prefix_seam = b->prefix_total + (n + 1);
    b->grid_node = dim3((unsigned)pn[n]);
    b->grid_sor = dim3((unsigned)ps[n]);
    b->grid_total = dim3((unsigned)pt[n]);
    b->grid_seam = dim3((unsigned)pm[n]);
    if (hipMemcpy(b->prefix_node, pn.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->prefix_sor, ps.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->prefix_total, pt.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->prefix_seam, pm.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice) != hipSuccess) {
        lbfd_batch_destroy(b);
        return LBFD_EHIP;
    }
    st = dispatch_for(p[0].lattice, p[0].precision).batch_table(b);
    if (st != LBFD_OK) {
        lbfd_batch_destroy(b);
        return st;
    }
    *out = b;
    return LBFD_OK;
}

lbfd_handle *lbfd_batch_instance(lbfd_batch *b, int32_t i)
{
    if (!b || i < 0 || i >= b->n) return nullptr;
    return b->inst[i];
}

int lbfd_batch_step(lbfd_batch *b, int64_t n)
{
    if (!b || n < 0) return LBFD_EINVAL;
    lbfd_handle *h0 = b->inst[0];
    bool dirty = false;
    for (lbfd_handle *h : b->inst) {
        if (h->step != h0->step || h->fc != h0->fc || h->pc != h0->pc || h->fd_hist != h0->fd_hist)
            return LBFD_EINVAL;
        dirty = dirty || h->kp_dirty;
    }
    Dispatch dp = dispatch_for(h0->p.lattice, h0->p.precision);
    if (dirty) {
        // a parameter block changed after the table was written (the buoyancy reference)
        if (hipStreamSynchronize(h0->stream) != hipSuccess) return LBFD_EHIP;
        const int st = dp.batch_table(b);
        if (st != LBFD_OK) return st;
        for (lbfd_handle *h : b->inst) h->kp_dirty = false;
        b->graphs.release();
    }
    return dp.batch_step(b, n);
}

// ------------------------------------------------------------------ frozen-flow substeps

int lbfd_write_field(lbfd_handle *h, int32_t field, const double *host, size_t count)
{
    if (!h) return LBFD_EINVAL;
    return dispatch_for(h->p.lattice, h->p.precision).write_field(h, field, host, count);
}

int lbfd_fd_substeps(lbfd_handle *h, int64_t k)
{
    if (!h || k < 0) return LBFD_EINVAL;
    return dispatch_for(h->p.lattice, h->p.precision).fd_substeps(h, k);
}

// ------------------------------------------------------------------ learned surrogate

struct lbfd_sg {
    lbfd_sg_params p;
    hipStream_t stream;
    sg::Net net;
    float *gflat;            // gradient in parameter order [n_params]
    double *loss;            // FP64 loss accumulator
    uint16_t *act[3];        // outputs of layers 1-3, BF16 [nodes][32]
    uint16_t *dy[2];         // gradients of layer outputs, BF16 [nodes][32]
    float *out;              // network output, FP32 [nodes][NOUT]
    uint16_t *feat;          // whole-field input grid, BF16 [nz+8][ny+8][nx+8][16]
    int *org;                // tile origins [3 max_batch]
    long long cap_act, cap_out, cap_feat;
    long long t;             // Adam steps taken
    bool wide = true;        // z-marching kernel on wide grids
    int cus = 256;           // compute units of the device (persistent grid of that kernel)
};

static long long cube(long long e) { return e * e * e; }

// Nodes of the outputs of layer l (1..4) for B grids of d x h x w input nodes.
static long long layer_nodes(int l, long long B, long long d, long long h, long long w)
{
    return B * (d - 2 * l) * (h - 2 * l) * (w - 2 * l);
}

struct SgLayout {
    size_t master, m, v, gflat, gw[sg::NL], gb[sg::NL], wb[sg::NL], wt[sg::NL], bias[sg::NL];
    size_t loss, act[3], dy[2], out, feat, org, total;
    long long cap_act, cap_out, cap_feat;
};

static int sg_layout(const lbfd_sg_params *p, SgLayout *L)
{
    if (!p || p->tile < 3 || p->tile > 64 || p->max_batch < 1 || p->k < 1) return LBFD_EINVAL;
    if (!(p->psi_inf > 0 && p->phi_s > 0 && p->u_s > 0 && p->dpsi_s > 0 && p->dphi_s > 0)) return LBFD_EINVAL;
    if (!(p->lr > 0 && p->beta1 >= 0 && p->beta1 < 1 && p->beta2 >= 0 && p->beta2 < 1 && p->adam_eps > 0))
        return LBFD_EINVAL;
    const bool field = p->field[0] > 0 || p->field[1] > 0 || p->field[2] > 0;
    if (field && (p->field[0] < 1 || p->field[1] < 1 || p->field[2] < 1)) return LBFD_EINVAL;
    const long long T = p->tile, B = p->max_batch;
    long long ca = layer_nodes(1, B, T + 8, T + 8, T + 8), co = B * cube(T), cf = 0;
    if (ca >= (1LL << 31)) return LBFD_EINVAL;   // node indices of a tile batch stay 32-bit
    if (field) {
        const long long fx = p->field[0] + 8, fy = p->field[1] + 8, fz = p->field[2] + 8;
        ca = std::max(ca, layer_nodes(1, 1, fz, fy, fx));
        co = std::max(co, layer_nodes(4, 1, fz, fy, fx));
        cf = fx * fy * fz;
    }
    if (ca * sg::CO * 2 > (1LL << 40)) return LBFD_EINVAL;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o += align256(b); return r; };
    const size_t np = (size_t)sg::n_params();
    L->master = take(4 * np);
    L->m = take(4 * np);
    L->v = take(4 * np);
    L->gflat = take(4 * np);
    for (int l = 0; l < sg::NL; ++l) {
        L->gw[l] = take(4 * 27 * sg::CIN_PAD[l] * sg::CO);
        L->gb[l] = take(4 * sg::CO);
        L->wb[l] = take(2 * 27 * sg::CIN_PAD[l] * sg::CO);
        L->wt[l] = take(2 * 27 * sg::CIN_PAD[l] * sg::CO);
        L->bias[l] = take(4 * sg::CO);
    }
    L->loss = take(8);
    for (int i = 0; i < 3; ++i) L->act[i] = take((size_t)ca * sg::CO * 2);
    for (int i = 0; i < 2; ++i) L->dy[i] = take((size_t)ca * sg::CO * 2);
    L->out = take((size_t)co * sg::NOUT * 4);
    L->feat = take((size_t)cf * sg::IN_CH * 2);
    L->org = take(sizeof(int) * 3 * (size_t)B);
    L->total = o;
    L->cap_act = ca;
    L->cap_out = co;
    L->cap_feat = cf;
    return LBFD_OK;
}

int64_t lbfd_sg_n_params(void) { return sg::n_params(); }

int lbfd_sg_workspace_bytes(const lbfd_sg_params *p, size_t *bytes)
{
    if (!bytes) return LBFD_EINVAL;
    SgLayout L;
    int st = sg_layout(p, &L);
    if (st != LBFD_OK) return st;
    *bytes = L.total;
    return LBFD_OK;
}

int lbfd_sg_create(const lbfd_sg_params *p, void *d_workspace, size_t bytes, void *stream, lbfd_sg **out)
{
    if (!out) return LBFD_EINVAL;
    *out = nullptr;
    SgLayout L;
    int st = sg_layout(p, &L);
    if (st != LBFD_OK) return st;
    if (!d_workspace || bytes < L.total || ((uintptr_t)d_workspace & 255) != 0) return LBFD_EWORKSPACE;
    lbfd_sg *s = new (std::nothrow) lbfd_sg();
    if (!s) return LBFD_ENOMEM;
    char *ws = (char *)d_workspace;
    s->p = *p;
    s->stream = (hipStream_t)stream;
    s->net.master = (float *)(ws + L.master);
    s->net.m = (float *)(ws + L.m);
    s->net.v = (float *)(ws + L.v);
    for (int l = 0; l < sg::NL; ++l) {
        s->net.gw[l] = (float *)(ws + L.gw[l]);
        s->net.gb[l] = (float *)(ws + L.gb[l]);
        s->net.wb[l] = (uint16_t *)(ws + L.wb[l]);
        s->net.wt[l] = (uint16_t *)(ws + L.wt[l]);
        s->net.bias[l] = (float *)(ws + L.bias[l]);
    }
    s->gflat = (float *)(ws + L.gflat);
    s->loss = (double *)(ws + L.loss);
    for (int i = 0; i < 3; ++i) s->act[i] = (uint16_t *)(ws + L.act[i]);
    for (int i = 0; i < 2; ++i) s->dy[i] = (uint16_t *)(ws + L.dy[i]);
    s->out = (float *)(ws + L.out);
    s->feat = (uint16_t *)(ws + L.feat);
    s->org = (int *)(ws + L.org);
    s->cap_act = L.cap_act;
    s->cap_out = L.cap_out;
    s->cap_feat = L.cap_feat;
    s->t = 0;
    {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            s->cus = n;
    }
    // weights, moments and the padded layouts start at zero
    if (hipMemsetAsync(ws, 0, L.loss, s->stream) != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess) {
        delete s;
        return LBFD_EHIP;
    }
    *out = s;
    return LBFD_OK;
}

void lbfd_sg_destroy(lbfd_sg *s)
{
    if (!s) return;
    hipStreamSynchronize(s->stream);
    delete s;
}

static int sg_pack(lbfd_sg *s, hipStream_t st, int adam)
{
    const double b1 = s->p.beta1, b2 = s->p.beta2;
    const float c1 = adam ? (float)(1.0 - std::pow(b1, (double)s->t)) : 1.0f;
    const float c2 = adam ? (float)(1.0 - std::pow(b2, (double)s->t)) : 1.0f;
    hipLaunchKernelGGL(sg::k_adam_pack, dim3((unsigned)((sg::n_params() + 255) / 256)), dim3(256), 0, st, s->net,
                       adam, (float)s->p.lr, (float)b1, (float)b2, (float)s->p.adam_eps, c1, c2);
    return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
}

int lbfd_sg_set_params(lbfd_sg *s, const float *host, int64_t n)
{
    if (!s || !host || n != sg::n_params()) return LBFD_EINVAL;
    const size_t b = sizeof(float) * (size_t)n;
    if (hipMemcpyAsync(s->net.master, host, b, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemsetAsync(s->net.m, 0, b, s->stream) != hipSuccess ||
        hipMemsetAsync(s->net.v, 0, b, s->stream) != hipSuccess)
        return LBFD_EHIP;
    s->t = 0;
    int st = sg_pack(s, s->stream, 0);
    if (st != LBFD_OK) return st;
    return hipStreamSynchronize(s->stream) == hipSuccess ? LBFD_OK : LBFD_EHIP;
}

int lbfd_sg_get_params(lbfd_sg *s, float *host, int64_t n)
{
    if (!s || !host || n != sg::n_params()) return LBFD_EINVAL;
    if (hipMemcpyAsync(host, s->net.master, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, s->stream) !=
            hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return LBFD_EHIP;
    return LBFD_OK;
}

static unsigned blocks_for(long long n, long long per) { return (unsigned)((n + per - 1) / per); }

// Output planes per column of the z-marching forward kernel.
constexpr int SG_ZC = 32;

// Forward pass over B grids of d x h x w input nodes on stream st; the layer
// outputs stay in s->act for a backward pass.
static int sg_forward_on(lbfd_sg *s, hipStream_t st, const uint16_t *in, int B, int d, int h, int w, float *out)
{
    if (!s || !in || !out || B < 1 || d < 9 || h < 9 || w < 9) return LBFD_EINVAL;
    const long long M1 = layer_nodes(1, B, d, h, w), M4 = layer_nodes(4, B, d, h, w);
    if (M1 > s->cap_act || M4 > s->cap_out) return LBFD_EINVAL;
    const void *x = in;
    for (int l = 0; l < sg::NL; ++l) {
        const int Di = d - 2 * l, Hi = h - 2 * l, Wi = w - 2 * l;
        const long long M = layer_nodes(l + 1, B, d, h, w);
        if (Wi - 2 >= 2 * sg::ZX && s->wide) {
            // wide grids: columns of 30 x 4 output nodes over SG_ZC planes, one persistent
            // workgroup per compute unit (the kernel's LDS and registers allow one)
            const int nbx = (Wi - 2 + sg::ZX - 1) / sg::ZX, nby = (Hi - 2 + sg::ZY - 1) / sg::ZY,
                      nbz = (Di - 2 + SG_ZC - 1) / SG_ZC;
            const long long ncol = (long long)nbx * nby * nbz * B;
            const dim3 grid((unsigned)std::min<long long>(ncol, s->cus));
            if (l == 0)
                hipLaunchKernelGGL((sg::k_conv_fwd_zm<16, true, false>), grid, dim3(256), 0, st, (const uint16_t *)x,
                                   s->net.wb[0], s->net.bias[0], (void *)s->act[0], Di, Hi, Wi, nbx, nby, nbz, SG_ZC,
                                   ncol);
            else if (l < 3)
                hipLaunchKernelGGL((sg::k_conv_fwd_zm<32, true, false>), grid, dim3(256), 0, st, (const uint16_t *)x,
                                   s->net.wb[l], s->net.bias[l], (void *)s->act[l], Di, Hi, Wi, nbx, nby, nbz, SG_ZC,
                                   ncol);
            else
                hipLaunchKernelGGL((sg::k_conv_fwd_zm<32, false, true>), grid, dim3(256), 0, st, (const uint16_t *)x,
                                   s->net.wb[3], s->net.bias[3], (void *)out, Di, Hi, Wi, nbx, nby, nbz, SG_ZC, ncol);
            if (l < 3) x = s->act[l];
            continue;
        }
        const dim3 grid(blocks_for(M, sg::FWD_NODES));
        if (l == 0)
            hipLaunchKernelGGL((sg::k_conv_fwd<16, true, false>), grid, dim3(256), 0, st, (const uint16_t *)x,
                               s->net.wb[0], s->net.bias[0], (void *)s->act[0], Di, Hi, Wi, M);
        else if (l < 3)
            hipLaunchKernelGGL((sg::k_conv_fwd<32, true, false>), grid, dim3(256), 0, st, (const uint16_t *)x,
                               s->net.wb[l], s->net.bias[l], (void *)s->act[l], Di, Hi, Wi, M);
        else
            hipLaunchKernelGGL((sg::k_conv_fwd<32, false, true>), grid, dim3(256), 0, st, (const uint16_t *)x,
                               s->net.wb[3], s->net.bias[3], (void *)out, Di, Hi, Wi, M);
        if (l < 3) x = s->act[l];
    }
    return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
}

int lbfd_sg_forward(lbfd_sg *s, const uint16_t *d_in, int32_t B, int32_t d, int32_t h, int32_t w, float *d_out)
{
    return sg_forward_on(s, s ? s->stream : nullptr, d_in, B, d, h, w, d_out);
}

// Loss and gradients of B training tiles (gradients in s->net.gw / gb).
static int sg_backward(lbfd_sg *s, const uint16_t *in, const float *tgt, int B)
{
    hipStream_t st = s->stream;
    const int E = s->p.tile + 8;
    int rc = sg_forward_on(s, st, in, B, E, E, E, s->out);
    if (rc != LBFD_OK) return rc;
    for (int l = 0; l < sg::NL; ++l) {
        if (hipMemsetAsync(s->net.gw[l], 0, sizeof(float) * 27 * sg::CIN_PAD[l] * sg::CO, st) != hipSuccess ||
            hipMemsetAsync(s->net.gb[l], 0, sizeof(float) * sg::CO, st) != hipSuccess)
            return LBFD_EHIP;
    }
    if (hipMemsetAsync(s->loss, 0, sizeof(double), st) != hipSuccess) return LBFD_EHIP;
    const long long M4 = layer_nodes(4, B, E, E, E);
    const long long T = s->p.tile;
    const float scale = (float)(2.0 / (2.0 * (double)B * (double)cube(T - 2)));
    hipLaunchKernelGGL(sg::k_cons_loss, dim3(std::min(1024u, blocks_for(M4, 256))), dim3(256), 0, st, s->out, tgt,
                       (int)T, M4, (float)(s->p.dpsi_s / s->p.dphi_s), scale, s->loss, s->dy[0]);
    int cur = 0;   // s->dy[cur]: gradient at the output of layer l + 1
    for (int l = sg::NL - 1; l >= 0; --l) {
        const int Di = E - 2 * l;
        const long long M = layer_nodes(l + 1, B, E, E, E);
        const uint16_t *x = l == 0 ? in : s->act[l - 1];
        const long long S = std::min<long long>(256, std::max<long long>(1, (M + 4095) / 4096));
        const long long per = ((M + S - 1) / S + 255) / 256 * 256;
        if (l == 0)
            hipLaunchKernelGGL((sg::k_conv_wgrad<16>), dim3(27, (unsigned)S), dim3(256), 0, st, x, s->dy[cur],
                               s->net.gw[l], s->net.gb[l], Di, Di, Di, M, per);
        else
            hipLaunchKernelGGL((sg::k_conv_wgrad<32>), dim3(27, (unsigned)S), dim3(256), 0, st, x, s->dy[cur],
                               s->net.gw[l], s->net.gb[l], Di, Di, Di, M, per);
        if (l > 0) {
            const long long Mi = layer_nodes(l, B, E, E, E);
            hipLaunchKernelGGL(sg::k_conv_dgrad, dim3(blocks_for(Mi, 256)), dim3(256), 0, st, s->dy[cur],
                               s->net.wt[l], s->act[l - 1], s->dy[1 - cur], Di, Di, Di, Mi);
            cur = 1 - cur;
        }
    }
    return hipGetLastError() == hipSuccess ? LBFD_OK : LBFD_EHIP;
}

static int sg_check_tiles(lbfd_sg *s, const uint16_t *in, const float *tgt, int B)
{
    if (!s || !in || !tgt || B < 1 || B > s->p.max_batch) return LBFD_EINVAL;
    return LBFD_OK;
}

int lbfd_sg_gradient(lbfd_sg *s, const uint16_t *d_in, const float *d_target, int32_t B, double *loss,
                     float *host_grad, int64_t n)
{
    int rc = sg_check_tiles(s, d_in, d_target, B);
    if (rc != LBFD_OK) return rc;
    if (!host_grad || n != sg::n_params()) return LBFD_EINVAL;
    rc = sg_backward(s, d_in, d_target, B);
    if (rc != LBFD_OK) return rc;
    hipLaunchKernelGGL(sg::k_grad_flat, dim3(blocks_for(sg::n_params(), 256)), dim3(256), 0, s->stream, s->net,
                       s->gflat);
    double L = 0.0;
    if (hipMemcpyAsync(host_grad, s->gflat, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, s->stream) !=
            hipSuccess ||
        hipMemcpyAsync(&L, s->loss, sizeof(double), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return LBFD_EHIP;
    const long long E = s->p.tile;
    if (loss) *loss = L / (2.0 * (double)B * (double)cube(E - 2));
    return LBFD_OK;
}

int lbfd_sg_train_step(lbfd_sg *s, const uint16_t *d_in, const float *d_target, int32_t B, double *loss)
{
    int rc = sg_check_tiles(s, d_in, d_target, B);
    if (rc != LBFD_OK) return rc;
    rc = sg_backward(s, d_in, d_target, B);
    if (rc != LBFD_OK) return rc;
    s->t += 1;
    rc = sg_pack(s, s->stream, 1);
    if (rc != LBFD_OK) return rc;
    if (loss) {
        double L = 0.0;
        if (hipMemcpyAsync(&L, s->loss, sizeof(double), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
            hipStreamSynchronize(s->stream) != hipSuccess)
            return LBFD_EHIP;
        *loss = L / (2.0 * (double)B * (double)cube(s->p.tile - 2));
    }
    return LBFD_OK;
}

static bool sg_periodic(const lbfd_handle *h)
{
    const int D = h->p.lattice == LBFD_D3Q19 ? 3 : 2;
    for (int a = 0; a < D; ++a)
        if (h->p.bc[a] != LBFD_PERIODIC) return false;
    return true;
}

static bool sg_fits_field(const lbfd_sg *s, const lbfd_handle *h)
{
    return h->p.nx <= s->p.field[0] && h->p.ny <= s->p.field[1] && h->p.nz <= s->p.field[2];
}

int lbfd_sg_features(lbfd_handle *h, lbfd_sg *s, uint16_t *d_feat)
{
    if (!h || !s || !d_feat || !sg_periodic(h)) return LBFD_EINVAL;
    return dispatch_for(h->p.lattice, h->p.precision)
        .sg_features(h, d_feat, (float)(1.0 / s->p.psi_inf), (float)(1.0 / s->p.phi_s), (float)(1.0 / s->p.u_s));
}

int lbfd_sg_snapshot(lbfd_handle *h, lbfd_sg *s, float *d_snap)
{
    if (!h || !s || !d_snap) return LBFD_EINVAL;
    return dispatch_for(h->p.lattice, h->p.precision).sg_snapshot(h, d_snap);
}

int lbfd_sg_tiles(lbfd_handle *h, lbfd_sg *s, const uint16_t *d_feat, const float *d_snap, const int32_t *host_org,
                  int32_t B, uint16_t *d_in, float *d_target)
{
    if (!h || !s || !d_feat || !d_snap || !host_org || !d_in || !d_target || B < 1 || B > s->p.max_batch)
        return LBFD_EINVAL;
    const int T = s->p.tile;
    for (int b = 0; b < B; ++b) {
        const int x = host_org[3 * b], y = host_org[3 * b + 1], z = host_org[3 * b + 2];
        if (x < 0 || y < 0 || z < 0 || x + T > h->p.nx || y + T > h->p.ny || z + T > h->p.nz) return LBFD_EINVAL;
    }
    if (hipMemcpyAsync(s->org, host_org, sizeof(int) * 3 * (size_t)B, hipMemcpyHostToDevice, h->stream) !=
        hipSuccess)
        return LBFD_EHIP;
    return dispatch_for(h->p.lattice, h->p.precision)
        .sg_tiles(h, d_feat, d_snap, s->org, B, T, d_in, d_target, (float)(1.0 / s->p.dpsi_s),
                  (float)(1.0 / s->p.dphi_s));
}

int lbfd_sg_set_drift_tol(lbfd_sg *s, double tol)
{
    if (!s || !(tol >= 0.0)) return LBFD_EINVAL;
    s->p.drift_tol = tol;
    return LBFD_OK;
}

int lbfd_sg_set_lr(lbfd_sg *s, double lr)
{
    if (!s || !(lr > 0.0) || !std::isfinite(lr)) return LBFD_EINVAL;
    s->p.lr = lr;
    return LBFD_OK;
}

int lbfd_sg_advance(lbfd_handle *h, lbfd_sg *s, int64_t nblocks, lbfd_sg_report *rep)
{
    if (!h || !s || nblocks < 0 || !h->p.fd_enable || !sg_periodic(h) || !sg_fits_field(s, h)) return LBFD_EINVAL;
    Dispatch dp = dispatch_for(h->p.lattice, h->p.precision);
    const int k = s->p.k;
    for (int64_t blk = 0; blk < nblocks; ++blk) {
        int rc = dp.sg_features(h, s->feat, (float)(1.0 / s->p.psi_inf), (float)(1.0 / s->p.phi_s),
                                (float)(1.0 / s->p.u_s));
        if (rc == LBFD_OK)
            rc = sg_forward_on(s, h->stream, s->feat, 1, h->p.nz + 8, h->p.ny + 8, h->p.nx + 8, s->out);
        if (rc == LBFD_OK) rc = dp.sg_candidate(h, s->out, (float)s->p.dpsi_s, (float)s->p.dphi_s);
        DevScalars sc;
        if (rc == LBFD_OK) rc = dp.read_scalars(h, &sc);
        if (rc != LBFD_OK) return rc;
        // the conservation check (the candidate's relative change of the total at the
        // frozen weights, before any rescaling) and the plausibility check
        const double drift = sc.drift_pre;
        const bool keep = std::isfinite(drift) && std::fabs(drift) <= s->p.drift_tol && sc.sg_bad == 0;
        rc = keep ? dp.sg_accept(h) : dp.fd_substeps(h, k);
        if (rc != LBFD_OK) return rc;
        if (rep) {
            rep->blocks += 1;
            rep->last_drift = drift;
            if (keep) {
                rep->accepted += 1;
                rep->max_drift = std::max(rep->max_drift, std::fabs(drift));
            } else {
                rep->fallbacks += 1;
            }
        }
        const bool was = h->fd_off;
        h->fd_off = true;
        rc = dp.step(h, k);
        h->fd_off = was;
        if (rc != LBFD_OK) return rc;
    }
    return LBFD_OK;
}

const char *lbfd_strerror(int s)
{
    switch (s) {
    case LBFD_OK: return "ok";
    case LBFD_EINVAL: return "invalid argument or parameter";
    case LBFD_ENOMEM: return "host allocation failed";
    case LBFD_EHIP: return "HIP runtime error";
    case LBFD_ENONFINITE: return "non-finite total surfactant";
    case LBFD_ESOR: return "SOR did not reach its tolerance within sor_max_sweeps";
    case LBFD_EWORKSPACE: return "device workspace missing, misaligned or too small";
    case LBFD_EUNSUPPORTED: return "unsupported combination";
    case LBFD_ESCRATCH: return "request larger than the library's fixed scratch buffer";
    default: return "unknown status";
    }
}

}  // extern "C"
