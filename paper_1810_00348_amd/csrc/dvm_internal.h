// Internal declarations shared by the kernels and the host runtime of
// libdvm_hip.so.  Not part of the public ABI (include/dvm.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dvm {

constexpr int NMOM = 13;     // raw velocity moments accumulated per cell
// stride of a partial record: 16 doubles = one 128-byte cache line, written
// whole by one store (the 3 slots past the moments take the reduction's
// unused sums), so that no line of the partials is ever partially written
constexpr int PREC = 16;
constexpr int PSTRIDE = 24;  // per-cell parameter slots
constexpr int MAXM = 512;    // velocity nodes per axis (upper bound)
constexpr int NKIND = 7;     // emission kinds: 6 box faces + the solid body

// per-cell equilibrium parameter slots (see params_kernel)
enum {
    P_NU = 0,   // 1/tau
    P_UX, P_UY, P_UZ,
    P_L0,       // 1 + lambda_0
    P_L1, P_L2, P_L3, P_L4,
    P_QX, P_QY, P_QZ,  // sigma * q (ES-BGK: the off-diagonal Lam^{-1} entries xy, xz, yz)
    P_TWO_T,    // 2 / T
    P_INFO,     // the cell info word (bit pattern in the slot's low 32 bits)
    P_IDX,      // 1 / cell size along x (non-uniform meshes)
    P_IDY,      // 1 / cell size along y
    P_NPARAM,
    P_RHO_SIDE = 16,  // 6 slots: inflow density of each side (wall rho_w or free-stream rho)
    P_IDZ = 22        // 1 / cell size along z
};

// cell info word: 4 bits per side (side s = 2 d + (upper ? 1 : 0)):
//   0       interior fluid neighbour
//   1..7    emission kind + 1 (0..5 box face, 6 solid body)
//   8       specular plane
// bit 24: the cell itself is solid
constexpr uint32_t SOLID_BIT = 1u << 24;
constexpr uint32_t CODE_SPECULAR = 8;

// lane table layout (doubles) per (octant, lane slot):
//   [0] xi_y [1] xi_z [2] a_y [3] a_z [4] b (y node) [5] c (z node)
//   then per velocity v of the lane: [6+4v] xi_x [7+4v] a_x [8+4v] w [9+4v] a (x node)
constexpr int LT_SHARED = 6;
constexpr int LT_PER_V = 4;

struct Consts {
    int nx, ny, nz, N;
    int mx, my, mz, MT, NV;
    double kappa_kn;      // kappa * Kn
    double omega, pr;
    int correct;
    int closed;
    int order2;           // second-order upwind: wall fluxes take the face values
    int esbgk;            // ES-BGK model in place of Shakhov's
    int xuniform;         // the x velocity axis is uniform (nodes a fixed step apart)
    double kind_rho[8];   // fixed emission density (free stream), per kind
    int kind_wall[8];     // 1: density from non-penetration
};

struct DevPtrs {
    const double* xi;     // [3][MAXM] axis nodes
    const double* wt;     // [3][MAXM] axis weights
    const double* xmom;   // [MAXM][5] x axis: w xi^p, p = 0..4
    const uint32_t* cellinfo;
    const int* bricks;    // int4 (I, J, K, 0) per brick, grouped by diagonal
    const double* lanetab;
    const double* h;      // cell sizes: [nx] along x, then [ny], then [nz]
};

template <typename S>
struct SweepArgs {
    const S* params;      // [N][PSTRIDE]
    const S* etab;        // [N][MT]: exp tables x | y | z (z scaled by nu * prefactor)
    const uint32_t* cellinfo;
    const S* ghat;        // [NKIND][NV] unit-density emission shapes
    const double* lanetab;
    const int* bricks;
    S* xface;
    S* yface;
    S* zface;
    S* spec;
    // second-order upwind: what each cell carries through its downstream
    // face (the linear extrapolation from it and its upwind neighbour),
    // beside the cell values of the faces and mirror planes above
    S* xgface;
    S* ygface;
    S* zgface;
    S* specg;
    double* partial;      // [8*ntiles][N][PREC]
    // second order on a stretched mesh: per axis (x, y, z) and direction
    // (+, -) the weight h_i / (h_i + h_upwind) of each cell index
    const double* theta;
    double rdx;           // 1 / h_x on a uniform mesh, 1 on a non-uniform one
    int nx, ny, nz, N, mx, my, MT, NV;
    int nbx, nby, nbz, bz;
    int ntiles, slots, lstride;
    int brick_off, brick_cnt;
    int oct_base, noct;
    int spec_on;
    int has_solid;
    int xuni;             // the x velocity axis is uniform (nodes a fixed step apart)
    int nblocks;
    // dependency-driven launches (sweep_kernel_dyn): ready flags
    // [8][ntiles][nbz][nby][nbx] holding the epoch of the launch that last
    // swept each brick, the work-unit counter and its value before this
    // launch, the number of work units, the failure flag word, and where the
    // launcher reports the number of waves it started (host memory)
    unsigned* ready;
    unsigned long long* head;
    unsigned long long qbase;
    unsigned epoch;
    int nitems;
    int* errflag;
    int* launched;
};

// kernel launchers (dvm_kernels.hip)
hipError_t launch_params(const Consts& C, const DevPtrs& D, const double* W, const double* q,
                         const double* rho_w, void* params, void* etab, int prec, int* flag,
                         hipStream_t st);
// ES-BGK parameters from the conserved moments and the stress per unit mass
hipError_t launch_params_es(const Consts& C, const DevPtrs& D, const double* W, const double* stress,
                            const double* rho_w, void* params, void* etab, int prec, int* flag, hipStream_t st);
hipError_t launch_emission(const Consts& C, const DevPtrs& D, const double* kind_state /*[NKIND][4]*/,
                           int nkind, void* ghat, double* ghat64, double* gout, int prec,
                           hipStream_t st);
hipError_t launch_wall_init(const Consts& C, const DevPtrs& D, const void* params, const void* etab,
                            const double* ghat64, const double* gout, double* rho_w, int prec,
                            hipStream_t st);
// wide_params: FP32 storage of f with the parameter record, Gaussian tables
// and equilibrium evaluation in FP64 (args' params and etab point to doubles)
hipError_t launch_sweep(int prec, int vl, int bx, int by, int pipelined, int nonuniform, int order2,
                        int esbgk, int wide_params, const void* args, hipStream_t st);
bool sweep_wide_params_available(int prec, int vl, int bx, int by, int nonuniform, int order2, int esbgk);
hipError_t launch_finalize(const Consts& C, const DevPtrs& D, const double* partial, int ntiles,
                           const double* gout, double* Wn, double* qn, double* rwn, double* stress_n,
                           double* blockmass, int nblocks, int* flag, hipStream_t st);
hipError_t launch_scale_residual(const Consts& C, const DevPtrs& D, double M0,
                                 const double* blockmass, int nbm, double* Wn, double* qn,
                                 double* rwn, const double* Wo, double* respart, int nblocks,
                                 hipStream_t st);
hipError_t launch_residual_final(const double* respart, int nblocks, const double* blockmass,
                                 int nbm, double* out, const int* flag, hipStream_t st);
// acc[o][cell] (= or +=) sum over the ntiles records partial[o*ntiles + t][cell]
hipError_t launch_fold(const double* partial, int ntiles, int N, int add, double* acc, hipStream_t st);
hipError_t launch_selftest_reduce(const double* in, double* out, hipStream_t st);
bool sweep_variant_available(int prec, int vl, int bx, int by, int nonuniform, int order2 = 0, int esbgk = 0);

}  // namespace dvm
