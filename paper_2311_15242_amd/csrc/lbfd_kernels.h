// lbfd_kernels.h -- HIP kernels (gfx950) of one time step of the hybrid
// lattice-Boltzmann colour-gradient / finite-difference surfactant method.
//
// State layout in HBM (structure of arrays, x fastest, node n = x + nx (y + ny z)):
//   f[2]      total populations f_i = f^R_i + f^B_i, Q planes, ping-pong
//   mac[2]    rho^R, rho^B, rhoN, j_x, j_y(, j_z) of a time level (j = sum f e)
//   desc[2]   per-node outflow descriptor written by the collision: colour share
//             a = rho^R/rho and recolouring vector c (D); in deviation modes also
//             rho and the post-collision velocity u* (D)
//   G[2]      |grad rhoN| of two time levels; nrm: interface normal (D)
//   u, F      fluid velocity (eq 10) and total force (D each)
//   psi[2], phi[2], Sprev, Bprev, rhsP, rhsF   finite-difference fields
//
// Only the total population is stored. Recolouring (eq 11) splits the
// post-collision f_dag_i of a node into a red part a f_dag_i + r_i and a blue
// part (1 - a) f_dag_i - r_i, where r_i is a closed form of node scalars; the
// macro kernel therefore rebuilds rho^R and rho^B of the next step from the
// streamed totals and the descriptors of the nodes they came from. This is the
// same arithmetic as propagating two colour populations, at half the bytes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbfd_lattice_tables.h"

namespace lbfd {

// ------------------------------------------------------------------ precision

struct PrecF64 { using R = double; using S = double; static constexpr bool DEV = false; };
struct PrecF32 { using R = float; using S = float; static constexpr bool DEV = false; };
struct PrecF16 { using R = float; using S = _Float16; static constexpr bool DEV = true; };
struct bf16 { uint16_t bits; };
struct PrecB16 { using R = float; using S = bf16; static constexpr bool DEV = true; };

__device__ __forceinline__ float to_real(bf16 v) { return __uint_as_float((uint32_t)v.bits << 16); }
__device__ __forceinline__ float to_real(_Float16 v) { return (float)v; }
__device__ __forceinline__ float to_real(float v) { return v; }
__device__ __forceinline__ double to_real(double v) { return v; }

template <class S> __device__ __forceinline__ S from_real(float v);
template <> __device__ __forceinline__ float from_real<float>(float v) { return v; }
template <> __device__ __forceinline__ _Float16 from_real<_Float16>(float v) { return (_Float16)v; }
template <> __device__ __forceinline__ bf16 from_real<bf16>(float v)
{
    // round to nearest even; finite inputs only (populations are finite)
    uint32_t u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return bf16{(uint16_t)(u >> 16)};
}
__device__ __forceinline__ double from_real_d(double v) { return v; }

// ------------------------------------------------------------------ lattices

template <int LAT> struct Lat;
template <> struct Lat<0> : D2Q9Tables {};
template <> struct Lat<1> : D3Q19Tables {};

// ------------------------------------------------------------------ parameters

constexpr int QMAX = 19;
constexpr int MAX_SWEEPS = 256;

// Device-resident scalars: the rescaling factor, the rescaling target, and the
// bookkeeping of the implicit solve and of error detection.
struct DevScalars {
    double scale;                 // stored psi, phi are multiplied by this on read
    double M0;                    // total surfactant to restore
    double Mlast;                 // total after the last solve, before rescaling
    double drift_pre;             // (Mlast - M0) / M0
    unsigned long long rmax[2];   // max |rhs| over active rows (bits of a non-negative double)
    unsigned long long res[2][MAX_SWEEPS];  // max |residual| per sweep
    int32_t sweeps[2];
    int32_t status;               // sticky lbfd_status of device-detected errors
    int32_t pad;
};

template <class R> struct Fields {
    void *f[2];
    R *mac[2];      // planes: 0 rhoR, 1 rhoB, 2 rhoN, 3.. j
    R *desc[2];     // planes: 0 a, 1.. c, then (deviation modes) rho, u*
    R *G[2];
    R *nrm;
    R *u;
    R *F;
    R *psi[2];
    R *phi[2];
    R *Sp, *Bp, *rhsP, *rhsF;
    double *part;   // reduction partials
    DevScalars *sc;
};

template <class R> struct KP {
    int nx, ny, nz;
    long long N;
    int bc[3];
    R wall_u[6][3];
    R rhoR0, rhoB0;
    R muR0, muB0;
    R alpha[2];         // sound-speed parameters alpha^k of red, blue (App. A, eq 42)
    R cs2[2];           // (cs^k)^2 of red, blue
    R qcoef[2];         // prefactor of the correction Q_a per colour
    int qon;            // correction present (some qcoef != 0)
    R rest[2][QMAX];    // rest equilibrium per unit density of each colour
    R beta;
    int recolour_literal;
    R sigma0, E0, psi_inf, sigma_min, cmc;
    R Ds, Db, ra, rd;
    int source_mode;
    R grav[3];
    R omega;
    R tol;
    R weno_eps, eps_n;
    R fd_eps;           // background support of the FD weights
    R upwind_eps;       // |u_a| band with upwind weights 1/2
    int rescale;
    // time-level selectors set per launch by the host
    int lev;            // mac/G/desc level of the current time n (n & 1)
    int fc;             // f buffer holding f^n
    int pc;             // psi/phi buffer holding the current values
    long long step;     // n
    Fields<R> fld;
};

// ------------------------------------------------------------------ indexing

struct Node { int x, y, z; bool ok; };

template <class R> __device__ __forceinline__ Node node_id(const KP<R> &k)
{
    Node n;
    n.x = blockIdx.x * blockDim.x + threadIdx.x;
    n.y = blockIdx.y * blockDim.y + threadIdx.y;
    n.z = blockIdx.z;
    n.ok = n.x < k.nx && n.y < k.ny;
    return n;
}

template <class R> __device__ __forceinline__ long long lin(const KP<R> &k, int x, int y, int z)
{
    return (long long)x + (long long)k.nx * ((long long)y + (long long)k.ny * z);
}

// Coordinate along one axis for stencils: periodic wrap, or the mirror image
// across a half-way wall (c = -1-j -> j, c = n+j -> n-1-j). |offset| <= 2.
__device__ __forceinline__ int fold(int c, int n, int wall, bool &mir)
{
    if (c >= 0 && c < n) return c;
    if (!wall) return c < 0 ? c + n : c - n;
    mir = true;
    return c < 0 ? -1 - c : 2 * n - 1 - c;
}

// Node index of (x,y,z)+(dx,dy,dz) and the sign of the odd_axis component of a
// vector field there (-1 when mirrored across a wall normal to that axis).
template <class R>
__device__ __forceinline__ long long nb(const KP<R> &k, int x, int y, int z, int dx, int dy, int dz, int odd_axis,
                                        R &sign)
{
    bool mx = false, my = false, mz = false;
    int X = fold(x + dx, k.nx, k.bc[0], mx);
    int Y = fold(y + dy, k.ny, k.bc[1], my);
    int Z = fold(z + dz, k.nz, k.bc[2], mz);
    bool flip = (odd_axis == 0 && mx) || (odd_axis == 1 && my) || (odd_axis == 2 && mz);
    sign = flip ? R(-1) : R(1);
    return lin(k, X, Y, Z);
}

// Isotropic lattice derivative (the stencil with which eq 9 evaluates every
// partial derivative): d_a chi = (1/cs^2) sum_i w_i e_ia chi(x + e_i), cs^2 = 1/3,
// summed over opposite pairs so that a uniform field gives an exact zero.
template <int LAT, class R>
__device__ __forceinline__ R lat_deriv(const KP<R> &k, const R *chi, R scl, int x, int y, int z, int a,
                                       int odd_axis)
{
    using L = Lat<LAT>;
    R acc = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        if (L::OPP[i] < i || L::E[i][a] == 0) continue;
        R s1, s2;
        long long p = nb(k, x, y, z, L::E[i][0], L::E[i][1], L::E[i][2], odd_axis, s1);
        long long m = nb(k, x, y, z, -L::E[i][0], -L::E[i][1], -L::E[i][2], odd_axis, s2);
        R d = s1 * chi[p] - s2 * chi[m];
        acc += R(L::W[i] * L::E[i][a]) * d;
    }
    return R(3) * acc * scl;
}

// Rest-plus-motion reference of a population leaving a node with density rho,
// colour share a and velocity us: rho [a phiR_i + (1-a) phiB_i + w_i (3 e.u + 4.5 (e.u)^2 - 1.5 u^2)].
// Deviation modes store f_i minus this, evaluated at the node the population left.
template <int LAT, class R>
__device__ __forceinline__ R reference(const KP<R> &k, int i, R rho, R a, const R *us)
{
    using L = Lat<LAT>;
    R eu = 0, uu = 0;
#pragma unroll
    for (int d = 0; d < L::D; ++d) { eu += R(L::E[i][d]) * us[d]; uu += us[d] * us[d]; }
    R rest = a * k.rest[0][i] + (R(1) - a) * k.rest[1][i];
    return rho * (rest + R(L::W[i]) * (R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu));
}

// Source node of the population arriving at (x,y,z) in direction j, and the
// direction it had when it left (a population that left through a wall comes
// back to the same node reversed: half-way bounce-back).
template <int LAT, class R>
__device__ __forceinline__ long long source_of(const KP<R> &k, int x, int y, int z, int j, int &pre)
{
    using L = Lat<LAT>;
    int c[3] = {x - L::E[j][0], y - L::E[j][1], z - L::E[j][2]};
    int lim[3] = {k.nx, k.ny, k.nz};
    bool wall = false;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (k.bc[a] && (c[a] < 0 || c[a] >= lim[a])) wall = true;
    if (wall) {
        pre = L::OPP[j];
        return lin(k, x, y, z);
    }
    pre = j;
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = c[a] < 0 ? c[a] + lim[a] : (c[a] >= lim[a] ? c[a] - lim[a] : c[a]);
    return lin(k, c[0], c[1], c[2]);
}

// Load the population j stored at node n (after propagation) as a real number,
// decoding a deviation with the descriptor of the node it came from.
template <int LAT, class P>
__device__ __forceinline__ typename P::R load_pop(const KP<typename P::R> &k, const typename P::S *f, long long n,
                                                  int j, long long src, const typename P::R *desc)
{
    using R = typename P::R;
    R v = to_real(f[(long long)j * k.N + n]);
    if constexpr (P::DEV) {
        using L = Lat<LAT>;
        const long long N = k.N;
        R us[3] = {0, 0, 0};
        R a = desc[src];
        R rho = desc[(1 + L::D) * N + src];
#pragma unroll
        for (int d = 0; d < L::D; ++d) us[d] = desc[(2 + L::D + d) * N + src];
        v += reference<LAT, R>(k, j, rho, a, us);
    }
    return v;
}

// ------------------------------------------------------------------ wave reductions

template <class T> __device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long *addr, double v)
{
    atomicMax(addr, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ double bits_to_double(unsigned long long b) { return __longlong_as_double((long long)b); }

}  // namespace lbfd
