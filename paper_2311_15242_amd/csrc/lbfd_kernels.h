// lbfd_kernels.h -- HIP kernels (gfx950) of one time step of the hybrid
// lattice-Boltzmann colour-gradient / finite-difference surfactant method.
//
// State layout in HBM (structure of arrays, x fastest, node n = x + nx (y + ny z)):
//   f[2]      total populations f_i = f^R_i + f^B_i, Q planes, ping-pong. In the
//             16-bit deviation modes the buffer holding the state between steps
//             stores non-equilibrium moments instead (load_moments), and the
//             propagated populations are 16-bit deviations from a reference
//             of the node they left (reference), converted back to moments in
//             place by the macro kernel
//   mac[2]    rho^R, rho^B, rhoN, j_x, j_y(, j_z) of a time level (j = sum f e)
//   desc      per-node outflow descriptor written by the collision, packed four
//             reals per node so that the macro kernel gathers it with one vector
//             load per source: colour share a = rho^R/rho and recolouring
//             vector c; in deviation modes also rho and the velocity u*
//   G[2]      |grad rhoN| of two time levels; nrm: interface normal (D)
//   u, F      fluid velocity (eq 10) and total force (D each)
//   qf        sum_k qcoef_k rho^k u_a (D), the field whose derivative is the
//             colour-summed correction Q_a
//   psi[2], phi[2], Sprev, Bprev   finite-difference fields (node order)
//   rhs2, cs2, cw2   the implicit solve's right-hand sides, iterates and node
//             weights as (psi, phi) pairs in colour-split order
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

// The FP16 mode stores its deviations and non-equilibrium moments scaled by
// 2^12: FP16 keeps 11 significant bits only above 2^-14 (6.1e-5), and
// deviations of slow or starting flows (1e-8 to 1e-5) would otherwise fall among
// the subnormals; scaled, they stay normal down to 1.5e-8 while the largest
// storable value is 16 (deviations and moments stay below 1). Powers of two
// scale exactly.
constexpr float F16_SCALE = 4096.0f, F16_ISCALE = 1.0f / 4096.0f;

__device__ __forceinline__ float to_real(bf16 v) { return __uint_as_float((uint32_t)v.bits << 16); }
__device__ __forceinline__ float to_real(_Float16 v) { return (float)v * F16_ISCALE; }
__device__ __forceinline__ float to_real(float v) { return v; }
__device__ __forceinline__ double to_real(double v) { return v; }

template <class S> __device__ __forceinline__ S from_real(float v);
template <> __device__ __forceinline__ float from_real<float>(float v) { return v; }
template <> __device__ __forceinline__ _Float16 from_real<_Float16>(float v) { return (_Float16)(v * F16_SCALE); }
template <> __device__ __forceinline__ bf16 from_real<bf16>(float v)
{
    // round to nearest even; finite inputs only (populations are finite)
    uint32_t u = __float_as_uint(v);
    u += 0x7fffu + ((u >> 16) & 1u);
    return bf16{(uint16_t)(u >> 16)};
}
__device__ __forceinline__ double from_real_d(double v) { return v; }

// Stochastic rounding of the BF16 stores of the deviation mode: a value between
// two BF16 neighbours is stored as the upper one with probability equal to its
// distance from the lower one over their spacing, so the stored value is exact
// on average. With round to nearest, a steady flow whose changes per step are
// below half a spacing of the stored deviations loses them at every step
// (stagnation); the error then repeats instead of averaging out and biases slow
// flows. r16 holds 16 uniform random bits; finite inputs only. The FP16 mode
// keeps round to nearest.
template <class S> __device__ __forceinline__ S from_real_sr(float v, uint32_t) { return from_real<S>(v); }
template <> __device__ __forceinline__ bf16 from_real_sr<bf16>(float v, uint32_t r16)
{
    return bf16{(uint16_t)((__float_as_uint(v) + r16) >> 16)};
}

// Random bits of the stochastic rounding: a 32-bit generator per node and
// stage, seeded by the lowbias32 integer hash (C. Wellons) of the node index,
// the step counter and the stage, then advanced by one linear congruential
// step (multiplier 747796405, increment 2891336453, as in PCG32) per value; the
// upper 16 bits are used. Deterministic: the same node, step and stage give the
// same bits in a single run, a batch and a graph replay.
struct Dither {
    uint32_t s;
    __device__ __forceinline__ Dither(uint32_t node, uint32_t tick, uint32_t stage)
    {
        uint32_t x = node * 0x9e3779b9u ^ (tick * 0x85ebca6bu + stage * 0xc2b2ae35u);
        x ^= x >> 16;
        x *= 0x7feb352du;
        x ^= x >> 15;
        x *= 0x846ca68bu;
        x ^= x >> 16;
        s = x;
    }
    __device__ __forceinline__ uint32_t next()
    {
        s = s * 747796405u + 2891336453u;
        return s >> 16;
    }
};

// ------------------------------------------------------------------ lattices

template <int LAT> struct Lat;
template <> struct Lat<0> : D2Q9Tables {};
template <> struct Lat<1> : D3Q19Tables {};

// Conserved moment rows (mass, momentum) of the moment bases: D2Q9 rows 0, 3, 5
// (eq 36), D3Q19 rows 0..3 (eq 39); state_slot numbers the remaining rows.
template <int LAT> __host__ __device__ constexpr bool conserved_row(int r)
{
    return LAT == 0 ? (r == 0 || r == 3 || r == 5) : r <= 3;
}
template <int LAT> __host__ __device__ constexpr int state_slot(int r)
{
    int s = 0;
    for (int i = 0; i < r; ++i) s += conserved_row<LAT>(i) ? 0 : 1;
    return s;
}

// Every moment row is a polynomial of one parity in e: M[r][opp(i)] = +M[r][i]
// for all i (even row) or -M[r][i] (odd row), and the columns of M^-1 follow
// the same parity. Opposite populations therefore enter an even row through
// f_i + f_opp(i) and an odd row through f_i - f_opp(i), which halves the
// products of the transforms.
template <int LAT> __host__ __device__ constexpr bool row_even(int r)
{
    using L = Lat<LAT>;
    for (int i = 0; i < L::Q; ++i)
        if (L::M[r][L::OPP[i]] != L::M[r][i]) return false;
    return true;
}
template <int LAT> constexpr bool rows_have_parity()
{
    using L = Lat<LAT>;
    for (int r = 0; r < L::Q; ++r) {
        const double sg = row_even<LAT>(r) ? 1.0 : -1.0;
        for (int i = 0; i < L::Q; ++i)
            if (L::M[r][L::OPP[i]] != sg * L::M[r][i] || L::MINV[L::OPP[i]][r] != sg * L::MINV[i][r]) return false;
    }
    return true;
}
static_assert(rows_have_parity<0>() && rows_have_parity<1>(), "moment rows without a definite parity");

// ------------------------------------------------------------------ parameters

constexpr int QMAX = 19;
constexpr int MAX_SWEEPS = 256;
constexpr int RSLOTS = 64;    // residual maxima of a sweep are spread over this many cache lines
constexpr int RSTRIDE = 16;   // 128 bytes between slots

// Device-resident scalars: the rescaling factor, the rescaling target, and the
// bookkeeping of the implicit solve and of error detection.
struct DevScalars {
    double scale;                 // stored psi, phi are multiplied by this on read
    double scale_prev;            // the factor of the other psi, phi buffer (previous time level)
    double M0;                    // total surfactant to restore
    double Mlast;                 // total after the last solve, before rescaling
    double drift_pre;             // (Mlast - M0) / M0
    unsigned long long rmax[2];   // max |rhs| of the last solve (bits of a non-negative double)
    int32_t sweeps[2];
    int32_t status;               // sticky lbfd_status of device-detected errors
    uint32_t tick;                // geometry launches since the state was set (one per step):
                                  // the time input of the stochastic rounding
    uint32_t sg_bad;              // nodes where a surrogate candidate changed psi or phi implausibly
    uint32_t sor_live;            // batched solve, sweeps past the third: systems of this instance
                                  // not yet converged before the coming half-sweep (bit 0 psi, bit 1 phi)
    double Mref;                  // total of the state a surrogate candidate starts from
};

// FP16 helpers of the packed descriptor (round to nearest even).
__device__ __forceinline__ float round_h(float v) { return (float)(_Float16)v; }
__device__ __forceinline__ uint32_t pack_h2(float lo, float hi)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)lo) |
           ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)hi) << 16);
}
__device__ __forceinline__ float h_lo(uint32_t v) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xffffu)); }
__device__ __forceinline__ float h_hi(uint32_t v) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16)); }

// Four reals read or written by one vector access (the packed descriptor).
template <class R> struct alignas(4 * sizeof(R)) V4 { R x, y, z, w; };
// A (psi, phi) pair of the implicit solve: one load serves both systems.
template <class R> struct alignas(2 * sizeof(R)) V2 { R x, y; };

// Recolouring descriptor of a node in the 16-bit deviation modes (16 bytes): colour
// share and density in FP32, the recolouring vector c and the reference velocity u*
// in FP16 (c_x, c_y | c_z, u*_x in 3-D; c_x, c_y | u*_x, u*_y in 2-D); u*_y, u*_z of
// 3-D lattices follow in a second plane. FP64 and FP32 modes use a V4 (a, c).
struct alignas(16) DescDev {
    float a, rho;
    uint32_t c01, c2u0;
};

template <class R> struct Fields {
    void *f[2];
    R *mac[2];      // planes: 0 rhoR, 1 rhoB, 2 rhoN, 3.. j
    void *desc;     // N x V4 (a, c) (FP64, FP32), or N x DescDev then N x 2 FP16 (deviation modes)
    R *G[2];
    R *nrm;
    R *u;
    R *F;
    R *qf;
    R *psi[2];
    R *phi[2];
    R *Sp, *Bp;
    // The implicit solve works on colour-split arrays (split_idx): right-hand
    // sides, iterates and node weights W = G + eps, X + eps of both systems
    V2<R> *rhs2, *cs2, *cw2;   // implicit solve: (psi, phi) pairs of right-hand sides, iterates, node weights
    double *part;   // reduction partials
    unsigned long long *sorres;  // residual and |rhs| maxima per field, sweep and slot (bits of doubles)
    DevScalars *sc;
};

template <class R> struct KP {
    int nx, ny, nz;
    int gx;             // tiles along x of the node launches (64 x each)
    int gy[3];          // tiles along y for workgroups of 1, 2 and 4 rows of 64 x
    long long N;
    int bc[3];
    R wall_u[6][3];
    R wterm[6][QMAX];   // 6 w_i (e_i . u_w) per wall (-x,+x,-y,+y,-z,+z) and direction
    int wmove;          // some wterm is nonzero (a wall moves)
    R rhoR0, rhoB0;
    R irho0[2];         // 1/rhoR0, 1/rhoB0
    R muR0, muB0;
    R ihmu[2];          // 1/(2 muR0), 1/(2 muB0)
    R alpha[2];         // sound-speed parameters alpha^k of red, blue (App. A, eq 42)
    R cs2[2];           // (cs^k)^2 of red, blue
    R qcoef[2];         // prefactor of the correction Q_a per colour
    int qon;            // correction present (some qcoef != 0)
    R rest[2][QMAX];    // rest equilibrium per unit density of each colour
    R beta;
    int recolour_literal;
    R sigma0, E0, psi_inf, sigma_min, cmc;
    double sigma0_d, E0_d, psi_inf_d, cmc_d;  // FP64 copies: the equation of state near saturation
    int eos_linear;     // sigma = sigma0 (1 - E0 psi / psi_inf) without a floor (Sec 3.2)
    R Ds, Db, ra, rd;
    int source_mode;
    R grav[3];
    R rho_ref;          // reference density of the buoyancy (rhoB0, or the domain mean)
    R omega;
    R tol;
    int seam;           // periodic axes of odd extent (bit a): seam classes of the SOR ordering
    double inv_hx, inv_ny;  // 1 / ((nx + 1) / 2) and 1 / ny for the SOR index arithmetic
    double inv_nx;          // 1 / nx
    uint32_t hx, hn;        // (nx + 1) / 2 and hx ny nz: row length and size of a colour plane
    int sor_exact;      // omega = 1 without seam classes: the red residual is the whole residual
    R weno_eps, eps_n;
    R fd_eps;           // background support of the FD weights
    R upwind_eps;       // |u_a| band with upwind weights 1/2
    int rescale;
    int extrap;         // a previous psi, phi level exists: extrapolate the solver's initial guess
    int nsweeps;        // SOR sweeps launched per step
    // time-level selectors set per launch by the host
    int lev;            // mac/G/desc level of the current time n (n & 1)
    int fc;             // f buffer holding f^n
    int pc;             // psi/phi buffer holding the current values
    long long step;     // n
    Fields<R> fld;
};

// ------------------------------------------------------------------ indexing

struct Node { int x, y, z; bool ok; };

// XCD-aware tile order. The hardware hands workgroup i of a launch to XCD
// i mod 8, and each XCD has its own L2. Renumbering the tiles so that XCD x
// processes one contiguous range of tile indices keeps the halo rows and
// planes that neighbouring tiles share inside one L2. A bijection of [0, n).
__device__ __forceinline__ int xcd_tile(int i, int n)
{
    const int q = n >> 3, r = n & 7, x = i & 7, l = i >> 3;
    return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// Node of this thread in tile t of the gx * gy * nz tiles of blockDim.x by
// blockDim.y nodes (x fastest).
// Tiles along y of a node launch whose workgroups have `rows` rows of 64 x
// (1, 2 or 4: the tile shape is a tuning choice; results do not depend on it).
template <class R> __device__ __forceinline__ int gy_of(const KP<R> &k, int rows)
{
    return rows == 4 ? k.gy[2] : rows == 2 ? k.gy[1] : k.gy[0];
}

template <class R> __device__ __forceinline__ Node node_at(const KP<R> &k, int t)
{
    Node n;
    const int bx = t % k.gx, r = t / k.gx;
    const int gy = gy_of(k, (int)blockDim.y);
    n.x = bx * blockDim.x + threadIdx.x;
    // node launches use workgroups of 64 x by 1, 2 or 4 rows, so a wavefront is one
    // row of 64 x: its y (and z) are the same in every lane, and held in scalar
    // registers the neighbourhood arithmetic along y and z runs once per wavefront
    n.y = __builtin_amdgcn_readfirstlane((r % gy) * (int)blockDim.y + (int)threadIdx.y);
    n.z = r / gy;
    n.ok = n.x < k.nx && n.y < k.ny;
    return n;
}

// Node of this thread in a 1-D launch over all tiles, in XCD-aware order.
template <class R> __device__ __forceinline__ Node node_id(const KP<R> &k)
{
    return node_at(k, xcd_tile((int)blockIdx.x, (int)gridDim.x));
}

// Time-level selectors shared by every instance of a batch at a step.
struct StepArgs {
    int lev, fc, pc, extrap;
    long long step;
};
// Tiles of 256 entries over one colour's index space ((nx + 1) / 2 x ny x nz);
// entries past a row's last same-colour node are skipped by the kernels.
__host__ __device__ inline int sor_tiles_of(int nx, int ny, int nz)
{
    const long long e = (long long)((nx + 1) / 2) * ny * nz;
    return (int)((e + 255) / 256);
}

// a / d for a < 2^32 and d >= 1 from inv = 1 / d in FP64: the rounded product
// is within a relative 2^-52 of a / d, which for a < 2^32 leaves its integer
// part at the quotient or one below it; one correction step makes it exact.
__device__ __forceinline__ uint32_t udiv(uint32_t a, uint32_t d, double inv)
{
    uint32_t q = (uint32_t)((double)a * inv);
    if (a - q * d >= d) ++q;
    return q;
}

template <class R> __device__ __forceinline__ StepArgs step_args(const KP<R> &k)
{
    StepArgs s;
    s.lev = k.lev;
    s.fc = k.fc;
    s.pc = k.pc;
    s.extrap = k.extrap;
    s.step = k.step;
    return s;
}

// Instance and local tile of this workgroup in a batched launch: the tiles of all
// instances are numbered consecutively (prefix[i] = first tile of instance i,
// prefix[ninst] = total), in XCD-aware order over the whole range.
__device__ __forceinline__ void batch_tile(const int *prefix, int ninst, int &inst, int &local)
{
    const int g = xcd_tile((int)blockIdx.x, (int)gridDim.x);
    int lo = 0, hi = ninst;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= g) lo = mid;
        else hi = mid;
    }
    inst = lo;
    local = g - prefix[lo];
}

template <class R> __device__ __forceinline__ long long lin(const KP<R> &k, int x, int y, int z)
{
    return (long long)x + (long long)k.nx * ((long long)y + (long long)k.ny * z);
}

// Second plane of the deviation-mode descriptor (u*_y, u*_z of 3-D lattices).
template <class R> __device__ __forceinline__ uint32_t *desc_dev_b(const KP<R> &k)
{
    return (uint32_t *)((DescDev *)k.fld.desc + k.N);
}

// Element idx of an array addressed as a uniform base pointer plus a 32-bit
// byte offset. This maps onto the scalar-base + vector-offset form of the
// global loads and stores, and one offset serves every array with the same
// element size. Requires idx * sizeof(T) < 2^32 (the host bounds the node count).
// Global address space of the device pass (the host pass parses these templates
// too and has no such address space).
#if defined(__HIP_DEVICE_COMPILE__)
#define LBFD_GLOBAL __attribute__((address_space(1)))
#else
#define LBFD_GLOBAL
#endif

// Element idx of a device array (a 32-bit byte offset from the base). Every
// array these kernels touch is in global memory; the access goes through a
// global-address-space pointer, so it is a global (not flat) access even when
// the base was itself loaded from memory (the instance table of a batch).
template <class T> __device__ __forceinline__ T ld(const T *base, uint32_t idx)
{
    typedef const LBFD_GLOBAL T GT;
    return *(GT *)((const LBFD_GLOBAL char *)base + idx * (uint32_t)sizeof(T));
}
template <class T> __device__ __forceinline__ void st(T *base, uint32_t idx, const T &v)
{
    typedef LBFD_GLOBAL T GT;
    *(GT *)((LBFD_GLOBAL char *)base + idx * (uint32_t)sizeof(T)) = v;
}

// The same through a base that has one value in every lane (a plane of a
// population array), pinned to scalar registers: otherwise the compiler may fold
// the plane offset into per-lane 64-bit address arithmetic. The access goes
// through a global-address-space pointer so it stays a global (not flat) one.
template <class T> __device__ __forceinline__ LBFD_GLOBAL char *scalar_base(const T *p)
{
    const unsigned long long v = (unsigned long long)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (LBFD_GLOBAL char *)(((unsigned long long)hi << 32) | lo);
}
template <class T> __device__ __forceinline__ T ldu(const T *base, uint32_t idx)
{
    typedef const LBFD_GLOBAL T GT;
    return *(GT *)(scalar_base(base) + idx * (uint32_t)sizeof(T));
}
template <class T> __device__ __forceinline__ void stu(T *base, uint32_t idx, const T &v)
{
    typedef LBFD_GLOBAL T GT;
    *(GT *)(scalar_base(base) + idx * (uint32_t)sizeof(T)) = v;
}

template <class R> __device__ __forceinline__ uint32_t node_index(const KP<R> &k, const Node &nd)
{
    return (uint32_t)nd.x + (uint32_t)k.nx * ((uint32_t)nd.y + (uint32_t)k.ny * (uint32_t)nd.z);
}

// Per-thread neighbourhood: for each axis a and offset o in {-2,-1,+1,+2} the
// linear index delta of the neighbour (periodic wrap, or the mirror image
// across a half-way wall: c = -1-j -> j, c = n+j -> n-1-j) and whether a wall
// was crossed. Computed once per node; every stencil, gather and push below
// is then a few integer adds.
struct Nbhd {
    int d[3][4];     // [axis][o + 2 for o<0, o + 1 for o>0]
    unsigned mir;    // bit a*4 + slot: the offset crossed a wall along axis a
};

__device__ __forceinline__ int slot_of(int o) { return o < 0 ? o + 2 : o + 1; }

template <class R> __device__ __forceinline__ Nbhd make_nbhd(const KP<R> &k, int x, int y, int z)
{
    Nbhd b;
    b.mir = 0u;
    const int c[3] = {x, y, z};
    const int n[3] = {k.nx, k.ny, k.nz};
    const int st[3] = {1, k.nx, k.nx * k.ny};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int sl = 0; sl < 4; ++sl) {
            const int o = sl < 2 ? sl - 2 : sl - 1;
            int t = c[a] + o;
            bool m = false;
            if (t < 0 || t >= n[a]) {
                if (k.bc[a]) { m = true; t = t < 0 ? -1 - t : 2 * n[a] - 1 - t; }
                else t = t < 0 ? t + n[a] : t - n[a];
            }
            b.d[a][sl] = (t - c[a]) * st[a];
            if (m) b.mir |= 1u << (a * 4 + sl);
        }
    }
    return b;
}

// Index delta of the neighbour at lattice offset (ex, ey, ez), each in {-2..2}.
__device__ __forceinline__ int nb_delta(const Nbhd &b, int ex, int ey, int ez)
{
    int d = 0;
    if (ex) d += b.d[0][slot_of(ex)];
    if (ey) d += b.d[1][slot_of(ey)];
    if (ez) d += b.d[2][slot_of(ez)];
    return d;
}

// Whether that offset crosses a wall along any axis, or along axis a.
__device__ __forceinline__ bool nb_wall(const Nbhd &b, int ex, int ey, int ez)
{
    unsigned m = 0u;
    if (ex) m |= (b.mir >> (0 * 4 + slot_of(ex))) & 1u;
    if (ey) m |= (b.mir >> (1 * 4 + slot_of(ey))) & 1u;
    if (ez) m |= (b.mir >> (2 * 4 + slot_of(ez))) & 1u;
    return m != 0u;
}

__device__ __forceinline__ bool nb_wall_axis(const Nbhd &b, int a, int ea)
{
    return ea != 0 && ((b.mir >> (a * 4 + slot_of(ea))) & 1u);
}

// Colour-split index of node (x, y, z) in the arrays of the implicit solve: each
// parity class (x + y + z) & 1 in a plane of its own, at (x >> 1) + hx (y + ny z).
// A colour half-sweep then reads and writes whole lines of its own plane and
// reads its face neighbours from whole lines of the other one.
template <class R> __device__ __forceinline__ uint32_t split_idx(const KP<R> &k, int x, int y, int z)
{
    return (uint32_t)((x + y + z) & 1) * k.hn + (uint32_t)(x >> 1) + k.hx * (uint32_t)(y + k.ny * z);
}

// Isotropic lattice derivative (the stencil with which eq 9 evaluates every
// partial derivative): d_a chi = (1/cs^2) sum_i w_i e_ia chi(x + e_i), cs^2 = 1/3,
// summed over opposite pairs so that a uniform field gives an exact zero.
// odd_axis >= 0 marks the odd_axis component of a vector field, which changes
// sign in a mirror normal to that axis.
template <int LAT, class R>
__device__ __forceinline__ R lat_deriv(const Nbhd &b, const R *chi, uint32_t n, R scl, int a, int odd_axis)
{
    using L = Lat<LAT>;
    R acc = 0;
#pragma unroll
    for (int i = 1; i < L::Q; ++i) {
        if (L::OPP[i] < i || L::E[i][a] == 0) continue;
        const int ex = L::E[i][0], ey = L::E[i][1], ez = L::E[i][2];
        R vp = ldu(chi, n + (uint32_t)nb_delta(b, ex, ey, ez));
        R vm = ldu(chi, n + (uint32_t)nb_delta(b, -ex, -ey, -ez));
        if (odd_axis >= 0) {
            const int eo = L::E[i][odd_axis];
            if (nb_wall_axis(b, odd_axis, eo)) vp = -vp;
            if (nb_wall_axis(b, odd_axis, -eo)) vm = -vm;
        }
        acc += R(L::W[i] * L::E[i][a]) * (vp - vm);
    }
    return R(3) * acc * scl;
}

// Rest-plus-motion reference of a population leaving a node with density rho,
// colour share a and velocity us: rho [a phiR_i + (1-a) phiB_i + w_i (3 e.u + 4.5 (e.u)^2 - 1.5 u^2)].
// Deviation modes store f_i minus this, evaluated at the node the population left.
// sgn = -1 evaluates it for the opposite direction of i (the rest weights and
// lattice weights are symmetric under e -> -e), which keeps every table index
// a compile-time constant.
template <int LAT, class R>
__device__ __forceinline__ R reference(const KP<R> &k, int i, R sgn, R rho, R a, const R *us)
{
    using L = Lat<LAT>;
    // zero components of e_i skipped: 0 * u and 0 + x are not folded in IEEE arithmetic
    R eu = 0, uu = us[0] * us[0];
    bool first = true;
#pragma unroll
    for (int d = 0; d < L::D; ++d) {
        if (d > 0) uu += us[d] * us[d];
        if (L::E[i][d] == 0) continue;
        eu = first ? R(L::E[i][d]) * us[d] : eu + R(L::E[i][d]) * us[d];
        first = false;
    }
    eu *= sgn;
    R rest = a * k.rest[0][i] + (R(1) - a) * k.rest[1][i];
    return rho * (rest + R(L::W[i]) * (R(3) * eu + R(4.5) * eu * eu - R(1.5) * uu));
}

// Moments of a second-order polynomial in e_i weighted by w_i:
// sum_i M_ri w_i [c0 + sum_a c1_a e_ia + sum_p c2_p (e_i e_i)_p], pairs p = xx yy zz xy xz yz
// (an off-diagonal coefficient multiplies e_ia e_ib once). Zero table entries fold away.
template <int LAT, class R> __device__ __forceinline__ R wpoly(int r, R c0, const R *c1, const R *c2)
{
    using L = Lat<LAT>;
    R v = 0;
    if (L::MW[r] != 0.0) v += R(L::MW[r]) * c0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (L::MWE[r][a] != 0.0) v += R(L::MWE[r][a]) * c1[a];
#pragma unroll
    for (int p = 0; p < 6; ++p)
        if (L::MWEE[r][p] != 0.0) v += R(L::MWEE[r][p]) * c2[p];
    return v;
}

// Reciprocal of a positive normal number: the hardware approximation (1 ulp) in
// FP32, the correctly rounded quotient in FP64.
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double fast_rcp(double x) { return 1.0 / x; }

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

// Slot of a maximum of field fi: index 2 s + colour for the pre-update residual of
// a half-sweep, RMAX_IDX for max |rhs|.
constexpr int RMAX_IDX = 2 * MAX_SWEEPS;
__device__ __forceinline__ unsigned long long *res_slot(unsigned long long *base, int fi, int idx, int slot)
{
    return base + ((size_t)(fi * (RMAX_IDX + 1) + idx) * RSLOTS + slot) * RSTRIDE;
}

// Block maxima of two non-negative values (a negative value means "nothing to
// record"), each folded into one of the RSLOTS slots of entry idx with one
// atomic per block. Every thread of the block must call it.
template <class R>
__device__ __forceinline__ void block_max_to_slots(R v0, R v1, unsigned long long *base, int idx)
{
    __shared__ double red[2][16];
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = t & 63, wv = t >> 6, nw = (blockDim.x * blockDim.y) >> 6;
    const double a = wave_max((double)v0), b = wave_max((double)v1);
    if (lane == 0) { red[0][wv] = a; red[1][wv] = b; }
    __syncthreads();
    if (t == 0) {
        double m[2] = {red[0][0], red[1][0]};
        for (int w = 1; w < nw; ++w) { m[0] = fmax(m[0], red[0][w]); m[1] = fmax(m[1], red[1][w]); }
        const int slot = (int)(blockIdx.x % RSLOTS);
#pragma unroll
        for (int fi = 0; fi < 2; ++fi)
            if (m[fi] >= 0.0) atomic_max_nonneg(res_slot(base, fi, idx, slot), m[fi]);
    }
    // thread 0 reads red above; a second call right after this one (the |rhs| maxima
    // of sweep 0) may overwrite it only once that read is done
    __syncthreads();
}

// Zero the slots of the 2 nsw half-sweeps and of max |rhs| (threads of one block).
__device__ __forceinline__ void sor_slots_clear(unsigned long long *base, int nsw)
{
    const int t = threadIdx.x + threadIdx.y * blockDim.x, nt = blockDim.x * blockDim.y;
    const int per = (2 * nsw + 1) * RSLOTS;
    for (int i = t; i < 2 * per; i += nt) {
        const int fi = i / per, r = i % per, e = r / RSLOTS, slot = r % RSLOTS;
        *res_slot(base, fi, e == 2 * nsw ? RMAX_IDX : e, slot) = 0ull;
    }
}

}  // namespace lbfd
