// HIP kernels (gfx950) of the iterative discrete-velocity scheme for the
// steady Shakhov model equation (arXiv:1810.00348, Secs. 2-3).
//
// Per outer iteration (eq. "iter_outer"):
//   params_kernel     per cell: U, T, 1/tau, Shakhov and conservative-correction
//                     parameters in FP64, and the three 1-D Gaussian factor
//                     tables of the Maxwellian (eqs. "feq", "mom", "mu_ref");
//                     params_es_kernel the same for the ES-BGK Gaussian, whose
//                     correction sums run over the whole velocity set per cell.
//   sweep_kernel_pf   the hot path: first-order upwind implicit sweep of every
//                     discrete velocity (eq. "sweeping_example") over 3-D bricks
//                     scheduled along brick diagonals (software-pipelined cell
//                     loop; sweep_kernel is the plain body, sweep_kernel_pfx the
//                     second-order and ES-BGK forms, sweep_kernel_dyn one
//                     dependency-driven launch), equilibrium evaluated on the
//                     fly, 13 raw moments reduced across the wave (eq. "macros")
//                     into deterministic per-tile partials.
//   finalize_kernel   per cell: sum of the partials, new conserved moments,
//                     heat flux about the new bulk velocity, wall densities from
//                     the non-penetration condition (eq. "rho_wall").
//   scale_residual /  closed-domain mass rescaling (Sec. 3.4) and the relative
//   residual_final    change of the conserved fields (Sec. 4.1).
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "dvm_internal.h"

namespace dvm {

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------

// Reciprocal of a positive normal number: hardware estimate refined by Newton
// steps (each squares the relative error: two for FP64, one for FP32; the
// FP32 estimate alone is biased enough to move the FP32 form's fixed point
// by 3-5x its rounding-level distance from the FP64 one).
__device__ __forceinline__ double fast_rcp(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ float fast_rcp(float d)
{
    const float r = __builtin_amdgcn_rcpf(d);
    const float e = fmaf(-d, r, 1.0f);
    return fmaf(r, e, r);
}

// reciprocals of a lane's VL denominators from one reciprocal of their
// product (products of the others: 3 (VL - 1) multiplications in place of
// VL - 1 reciprocals with their Newton steps)
template <int VL>
__device__ __forceinline__ void batch_rcp(const double (&d)[VL], double (&r)[VL])
{
    if constexpr (VL == 1) {
        r[0] = fast_rcp(d[0]);
    } else if constexpr (VL == 2) {
        const double q = fast_rcp(d[0] * d[1]);
        r[0] = q * d[1];
        r[1] = q * d[0];
    } else {
        static_assert(VL == 4, "batch_rcp: 1, 2 or 4 values");
        const double p01 = d[0] * d[1], p23 = d[2] * d[3];
        const double q = fast_rcp(p01 * p23);
        const double q01 = q * p23, q23 = q * p01;  // 1 / p01, 1 / p23
        r[0] = q01 * d[1];
        r[1] = q01 * d[0];
        r[2] = q23 * d[3];
        r[3] = q23 * d[2];
    }
}

// 5x5 symmetric positive definite solve by Cholesky (FP64).
__device__ bool chol5_solve(double A[5][5], const double b[5], double x[5])
{
    double L[5][5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int j = 0; j < 5; ++j) L[i][j] = 0.0;
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            double s = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 0.0)) return false;
                L[i][i] = sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    }
    double y[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
#pragma unroll
    for (int i = 4; i >= 0; --i) {
        double s = y[i];
#pragma unroll
        for (int k = i + 1; k < 5; ++k) s -= L[k][i] * x[k];
        x[i] = s / L[i][i];
    }
    return true;
}

// Correction multipliers from separable 1-D moments.
//   Mx[p] = sum_a w_a (xi_a - Ux)^p exp(-(xi_a - Ux)^2 / T), p = 0..5 (same y, z),
// so that sum over the grid of w c^(p,q,r) f^M = pre * Mx[p] My[q] Mz[r].
// Basis phi = (1, cx, cy, cz, |c|^2).  Solves A lam = t - sum w phi f^S with
// A_lk = sum w phi_l phi_k f^M and targets t = (rho, 0, 0, 0, 3 rho T / 2):
// the corrected equilibrium f^S + f^M lam.phi has exactly the discrete mass,
// momentum and energy of the state it is built from.
__device__ bool correction_lambda(const double Mx[6], const double My[6], const double Mz[6],
                                  double pre, double rho, double T, double sig, double qx,
                                  double qy, double qz, double lam[5])
{
    // monomials of phi_l: up to three exponent triples each
    const int nmon[5] = {1, 1, 1, 1, 3};
    const int ex[5][3][3] = {
        {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}},
        {{1, 0, 0}, {0, 0, 0}, {0, 0, 0}},
        {{0, 1, 0}, {0, 0, 0}, {0, 0, 0}},
        {{0, 0, 1}, {0, 0, 0}, {0, 0, 0}},
        {{2, 0, 0}, {0, 2, 0}, {0, 0, 2}},
    };
    auto mom = [&](int p, int q, int r) { return pre * Mx[p] * My[q] * Mz[r]; };
    double A[5][5], b[5];
    const double qv[3] = {qx, qy, qz};
    const double two_T = 2.0 / T;
#pragma unroll
    for (int l = 0; l < 5; ++l) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            double s = 0.0;
            for (int u = 0; u < nmon[l]; ++u)
                for (int v = 0; v < nmon[k]; ++v)
                    s += mom(ex[l][u][0] + ex[k][v][0], ex[l][u][1] + ex[k][v][1],
                             ex[l][u][2] + ex[k][v][2]);
            A[l][k] = s;
        }
        // sum w phi_l f^S = sum w phi_l f^M [1 + sig (c.q)(2|c|^2/T - 5)]
        double s = 0.0;
        for (int u = 0; u < nmon[l]; ++u) {
            const int p0 = ex[l][u][0], q0 = ex[l][u][1], r0 = ex[l][u][2];
            s += mom(p0, q0, r0);
            for (int d = 0; d < 3; ++d) {
                int pd = p0 + (d == 0), qd = q0 + (d == 1), rd = r0 + (d == 2);
                double t = -5.0 * mom(pd, qd, rd);
                t += two_T * (mom(pd + 2, qd, rd) + mom(pd, qd + 2, rd) + mom(pd, qd, rd + 2));
                s += sig * qv[d] * t;
            }
        }
        b[l] = -s;
    }
    b[0] += rho;
    b[4] += 1.5 * rho * T;
    return chol5_solve(A, b, lam);
}

// --------------------------------------------------------------------------
// A1: per-cell parameters
// --------------------------------------------------------------------------

template <typename S>
__device__ __forceinline__ S info_bits(uint32_t info)
{
    // the info word as the bit pattern of a record slot (its low 32 bits)
    if constexpr (sizeof(S) == 8)
        return __hiloint2double(0, (int)info);
    else
        return __int_as_float((int)info);
}

// One wave per 64 consecutive cells, one lane per cell.  A cell's record
// (PSTRIDE slots) and Gaussian tables (MT entries) are rows; the wave stages
// its rows in LDS and writes them out with consecutive lanes on consecutive
// entries, 32 table entries of an axis at a time, so that every store
// instruction covers whole cache lines (a lane writing its own row would
// touch 64 lines per instruction).  Solid cells get the info word and zeros.
constexpr int PCH = 32;  // table entries per staged chunk
template <typename S>
__global__ __launch_bounds__(64) void params_kernel(Consts C, DevPtrs D, const double* __restrict__ W,
                                                    const double* __restrict__ q,
                                                    const double* __restrict__ rho_w, S* __restrict__ params,
                                                    S* __restrict__ etab, int* __restrict__ flag)
{
    __shared__ S stage[64 * (PCH + 1)];
    static_assert(PCH + 1 >= PSTRIDE, "a record fits a staged row");
    const int lane = threadIdx.x;
    const int N = C.N;
    const int c0 = blockIdx.x * 64;
    const int nrow = min(64, N - c0);
    const int cell = c0 + lane;
    const bool live = lane < nrow;
    const uint32_t info = live ? D.cellinfo[cell] : SOLID_BIT;
    const bool fluid = !(info & SOLID_BIT);
    S rec[PSTRIDE];
#pragma unroll
    for (int k = 0; k < PSTRIDE; ++k) rec[k] = (S)0;
    rec[P_INFO] = info_bits<S>(info);
    bool eq = false;  // the equilibrium parameters are computed
    double rho = 1.0, Ux = 0.0, Uy = 0.0, Uz = 0.0, T = 1.0;
    if (fluid) {
        // inverse cell sizes (the upwind coefficients |xi_d| / h_d of a
        // non-uniform mesh)
        const int i = cell % C.nx, j = (cell / C.nx) % C.ny, k = cell / (C.nx * C.ny);
        rec[P_IDX] = (S)(1.0 / D.h[i]);
        rec[P_IDY] = (S)(1.0 / D.h[C.nx + j]);
        rec[P_IDZ] = (S)(1.0 / D.h[C.nx + C.ny + k]);
        // inflow density of each side: the wall density of iteration n at a
        // diffuse wall, the free-stream density at a free-stream face
        for (int sd = 0; sd < 6; ++sd) {
            const uint32_t code = (info >> (4 * sd)) & 15u;
            double rf = 0.0;
            if (code != 0 && code != CODE_SPECULAR)
                rf = C.kind_wall[code - 1] ? rho_w[(size_t)sd * N + cell] : C.kind_rho[code - 1];
            rec[P_RHO_SIDE + sd] = (S)rf;
        }
        rho = W[cell];
        Ux = W[N + cell] / rho;
        Uy = W[2 * N + cell] / rho;
        Uz = W[3 * N + cell] / rho;
        T = (W[4 * N + cell] - 0.5 * rho * (Ux * Ux + Uy * Uy + Uz * Uz)) / (0.75 * rho);
        eq = rho > 0.0 && T > 0.0 && isfinite(Ux) && isfinite(Uy) && isfinite(Uz) && isfinite(T);
        if (!eq) {
            // neutral equilibrium parameters (zero tables); the info word,
            // inverse sizes and inflow densities stay
            atomicOr(flag, 1);
            rec[P_NU] = (S)1;
        }
    }
    double qx = 0.0, qy = 0.0, qz = 0.0, nu = 0.0, pre = 0.0, sig = 0.0, invT = 1.0;
    if (eq) {
        qx = q[cell];
        qy = q[N + cell];
        qz = q[2 * N + cell];
        nu = rho * pow(T, 1.0 - C.omega) / C.kappa_kn;
        pre = rho * pow(M_PI * T, -1.5);
        sig = (1.0 - C.pr) * 4.0 / (5.0 * rho * T * T);
        invT = 1.0 / T;
    }
    double Mx[6], My[6], Mz[6];
    const double U3[3] = {Ux, Uy, Uz};
    const int m3[3] = {C.mx, C.my, C.mz};
    const int ce = lane & (PCH - 1), half = lane / PCH;
    int off = 0;
    for (int d = 0; d < 3; ++d) {
        double* M = d == 0 ? Mx : d == 1 ? My : Mz;
        for (int p = 0; p < 6; ++p) M[p] = 0.0;
        const double scale = d == 2 ? nu * pre : 1.0;
        const double* xi = D.xi + d * MAXM;
        const double* wt = D.wt + d * MAXM;
        for (int a0 = 0; a0 < m3[d]; a0 += PCH) {
            const int len = min(PCH, m3[d] - a0);
            for (int e = 0; e < len; ++e) {
                const int a = a0 + e;
                S ev = (S)0;
                if (eq) {
                    const double c = xi[a] - U3[d];
                    const double g = exp(-c * c * invT);
                    ev = (S)(g * scale);
                    double t = wt[a] * g;
#pragma unroll
                    for (int p = 0; p < 6; ++p) {
                        M[p] += t;
                        t *= c;
                    }
                }
                stage[lane * (PCH + 1) + e] = ev;
            }
            __syncthreads();
            if (ce < len) {
                for (int r = half; r < nrow; r += 64 / PCH)
                    etab[(size_t)(c0 + r) * C.MT + off + a0 + ce] = stage[r * (PCH + 1) + ce];
            }
            __syncthreads();
        }
        off += m3[d];
    }
    if (eq) {
        double lam[5] = {0, 0, 0, 0, 0};
        if (C.correct) {
            if (!correction_lambda(Mx, My, Mz, pre, rho, T, sig, qx, qy, qz, lam)) {
                atomicOr(flag, 2);
            }
        }
        rec[P_NU] = (S)nu;
        rec[P_UX] = (S)Ux;
        rec[P_UY] = (S)Uy;
        rec[P_UZ] = (S)Uz;
        rec[P_L0] = (S)(1.0 + lam[0]);
        rec[P_L1] = (S)lam[1];
        rec[P_L2] = (S)lam[2];
        rec[P_L3] = (S)lam[3];
        rec[P_L4] = (S)lam[4];
        rec[P_QX] = (S)(sig * qx);
        rec[P_QY] = (S)(sig * qy);
        rec[P_QZ] = (S)(sig * qz);
        rec[P_TWO_T] = (S)(2.0 * invT);
    }
    // the block's records are one contiguous run of nrow * PSTRIDE slots
#pragma unroll
    for (int k = 0; k < PSTRIDE; ++k) stage[lane * PSTRIDE + k] = rec[k];
    __syncthreads();
    S* out = params + (size_t)c0 * PSTRIDE;
    for (int idx = lane; idx < nrow * PSTRIDE; idx += 64) out[idx] = stage[idx];
}

hipError_t launch_params(const Consts& C, const DevPtrs& D, const double* W, const double* q,
                         const double* rho_w, void* params, void* etab, int prec, int* flag,
                         hipStream_t st)
{
    // one wave per 64 cells (the kernel stages its rows in LDS per wave)
    const int nb = (C.N + 63) / 64;
    if (prec == 0)
        params_kernel<double><<<nb, 64, 0, st>>>(C, D, W, q, rho_w, (double*)params, (double*)etab, flag);
    else
        params_kernel<float><<<nb, 64, 0, st>>>(C, D, W, q, rho_w, (float*)params, (float*)etab, flag);
    return hipGetLastError();
}

__device__ __forceinline__ double wave_reduce16(const double v[16]);

__device__ __forceinline__ double readlane_d(double x, int l)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// a lane that holds the sum of value k after wave_reduce16 (lane 16 r + 4 b
// holds value 4 bitreverse2(b) + bitreverse2(r))
__host__ __device__ constexpr int reduce16_lane(int k)
{
    return 16 * (((k & 1) << 1) | ((k >> 1) & 1)) + 4 * ((((k >> 2) & 1) << 1) | (k >> 3));
}

// ES-BGK (the ellipsoidal statistical model; the scheme applies to model
// equations other than Shakhov's, Sec. 2.1).  In the normalised units
// (R T = T/2) the target is the Gaussian
//   G = rho (2 pi)^{-3/2} det(Lam)^{-1/2} exp(-c^T Lam^{-1} c / 2),
//   Lam = (T/2) I / Pr + (1 - 1/Pr) Theta,  Theta = the stress per unit mass,
// relaxing with frequency Pr p / mu.  Its diagonal factors go to the tables
// (z scaled by nu * prefactor); the off-diagonal entries of Lam^{-1} to the
// cell record, for the cross factor exp(-(A_xy cx cy + A_xz cx cz + A_yz cy cz))
// the sweep takes per point.  The correction multipliers need the discrete
// moments of G, which does not factor over the axes: one pass over the whole
// velocity set per cell, shared by a wave (on a uniform x axis two products
// and five FMAs per node against the axis's w xi^p).
template <typename S>
__global__ __launch_bounds__(64) void params_es_kernel(Consts C, DevPtrs D, const double* __restrict__ W,
                                                       const double* __restrict__ stress,
                                                       const double* __restrict__ rho_w,
                                                       S* __restrict__ params, S* __restrict__ etab,
                                                       int* __restrict__ flag)
{
    // one wave per cell: the lanes share the pass over the velocity set
    const int cell = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t info = D.cellinfo[cell];
    S* P = params + (size_t)cell * PSTRIDE;
    if (lane == 0) reinterpret_cast<uint32_t*>(P + P_INFO)[0] = info;
    if (info & SOLID_BIT) return;
    if (lane == 0) {
        const int i = cell % C.nx, j = (cell / C.nx) % C.ny, k = cell / (C.nx * C.ny);
        P[P_IDX] = (S)(1.0 / D.h[i]);
        P[P_IDY] = (S)(1.0 / D.h[C.nx + j]);
        P[P_IDZ] = (S)(1.0 / D.h[C.nx + C.ny + k]);
        for (int s = 0; s < 6; ++s) {
            const uint32_t code = (info >> (4 * s)) & 15u;
            double rf = 0.0;
            if (code != 0 && code != CODE_SPECULAR)
                rf = C.kind_wall[code - 1] ? rho_w[(size_t)s * C.N + cell] : C.kind_rho[code - 1];
            P[P_RHO_SIDE + s] = (S)rf;
        }
    }
    const int N = C.N;
    S* E = etab + (size_t)cell * C.MT;
    const double rho = W[cell];
    const double Ux = W[N + cell] / rho, Uy = W[2 * N + cell] / rho, Uz = W[3 * N + cell] / rho;
    const double T = (W[4 * N + cell] - 0.5 * rho * (Ux * Ux + Uy * Uy + Uz * Uz)) / (0.75 * rho);
    // Lam = (T/2) I / Pr + (1 - 1/Pr) Theta, in (xx, yy, zz, xy, xz, yz) order
    double L[6];
    for (int k = 0; k < 6; ++k) L[k] = (1.0 - 1.0 / C.pr) * stress[(size_t)k * N + cell];
    for (int k = 0; k < 3; ++k) L[k] += 0.5 * T / C.pr;
    // inverse through the adjugate of [[a d e] [d b f] [e f c]]
    const double a = L[0], b = L[1], c = L[2], d = L[3], e = L[4], f = L[5];
    const double ca = b * c - f * f, cb = a * c - e * e, cc = a * b - d * d;
    const double cd = e * f - d * c, ce = d * f - e * b, cf = d * e - a * f;
    const double det = a * ca + d * cd + e * ce;
    if (!(rho > 0.0) || !(T > 0.0) || !isfinite(Ux) || !isfinite(Uy) || !isfinite(Uz) || !isfinite(T) ||
        !(det > 0.0) || !(ca > 0.0) || !(cc > 0.0)) {
        if (lane == 0) {
            atomicOr(flag, 1);
            for (int k = 0; k < P_INFO; ++k) P[k] = (S)0;
            P[P_NU] = (S)1;
        }
        for (int k = lane; k < C.MT; k += 64) E[k] = (S)0;
        return;
    }
    const double Axx = ca / det, Ayy = cb / det, Azz = cc / det;
    const double Axy = cd / det, Axz = ce / det, Ayz = cf / det;
    const double nu = C.pr * rho * pow(T, 1.0 - C.omega) / C.kappa_kn;
    const double pre = rho * pow(2.0 * M_PI, -1.5) / sqrt(det);
    for (int k = lane; k < C.MT; k += 64) {
        const int dd = k < C.mx ? 0 : k < C.mx + C.my ? 1 : 2;
        const int q = k - (dd == 0 ? 0 : dd == 1 ? C.mx : C.mx + C.my);
        const double Ad = dd == 0 ? Axx : dd == 1 ? Ayy : Azz;
        const double Ud = dd == 0 ? Ux : dd == 1 ? Uy : Uz;
        const double cq = D.xi[dd * MAXM + q] - Ud;
        E[k] = (S)((dd == 2 ? nu * pre : 1.0) * exp(-0.5 * Ad * cq * cq));
    }
    double lam[5] = {0, 0, 0, 0, 0};
    if (C.correct) {
        // discrete moments of G against the basis (1, cx, cy, cz, |c|^2);
        // lane l takes the (y, z) rows l, l + 64, ...
        double sm[14];
        for (int k = 0; k < 14; ++k) sm[k] = 0.0;
        // On a uniform x axis the exponent q(a) = Axx cx^2 / 2 + cx B + row is
        // quadratic in the node index, so exp(-q) follows from two products
        // per node: g(a+1) = g(a) r(a), r(a+1) = r(a) s with s = exp(-Axx h^2)
        // -- used on a row when neither end's exp(-q) nor any step factor
        // leaves the double range (else one exponential per node).
        const double hx = C.xuniform ? D.xi[1] - D.xi[0] : 0.0;
        const double sx = exp(-Axx * hx * hx);
        for (int r = lane; r < C.my * C.mz; r += 64) {
            const int ky = r % C.my, kz = r / C.my;
            const double cz = D.xi[2 * MAXM + kz] - Uz;
            const double cy = D.xi[MAXM + ky] - Uy;
            const double wyz = D.wt[MAXM + ky] * D.wt[2 * MAXM + kz];
            const double row = 0.5 * Ayy * cy * cy + 0.5 * Azz * cz * cz + Ayz * cy * cz;
            const double B = Axy * cy + Axz * cz;
            const double cyz2 = cy * cy + cz * cz;
            const double c0 = D.xi[0] - Ux, c1 = D.xi[C.mx - 1] - Ux;
            const double q0 = 0.5 * Axx * c0 * c0 + c0 * B + row;
            const double q1 = 0.5 * Axx * c1 * c1 + c1 * B + row;
            const double d0 = Axx * hx * (c0 + 0.5 * hx) + hx * B;  // q(1) - q(0)
            const double d1 = d0 + Axx * hx * hx * (C.mx - 2);      // q(M-1) - q(M-2)
            const bool rec = C.xuniform && fabs(q0) < 600.0 && fabs(q1) < 600.0 && fabs(d0) < 600.0 &&
                             fabs(d1) < 600.0;
            // the row's raw sums R_p = sum of w e xi_x^p, p = 0..4 (the axis's
            // w xi^p from a table), then taken about U_x; the y and z factors
            // of the monomials are applied once per row
            double R0 = 0, R1 = 0, R2 = 0, R3 = 0, R4 = 0;
            // the table through the constant address space: one scalar load
            // for the wave (the address is the same on every lane)
            using CT = const __attribute__((address_space(4))) double;
            CT* xm = (CT*)D.xmom;
            if (rec) {
                double g = exp(-q0), rr = exp(-d0);
#pragma unroll 4
                for (int kx = 0; kx < C.mx; ++kx) {
                    CT* t = xm + 5 * kx;
                    const double e = g;
                    g *= rr;
                    rr *= sx;
                    R0 = fma(t[0], e, R0);
                    R1 = fma(t[1], e, R1);
                    R2 = fma(t[2], e, R2);
                    R3 = fma(t[3], e, R3);
                    R4 = fma(t[4], e, R4);
                }
            } else {
                for (int kx = 0; kx < C.mx; ++kx) {
                    CT* t = xm + 5 * kx;
                    const double cx = D.xi[kx] - Ux;
                    const double e = exp(-(0.5 * Axx * cx * cx + cx * B + row));
                    R0 = fma(t[0], e, R0);
                    R1 = fma(t[1], e, R1);
                    R2 = fma(t[2], e, R2);
                    R3 = fma(t[3], e, R3);
                    R4 = fma(t[4], e, R4);
                }
            }
            // sum of w e (xi - U)^p = sum over j of C(p, j) (-U)^(p-j) R_j
            const double u1 = -Ux, u2 = u1 * u1, u3 = u2 * u1, u4 = u2 * u2;
            double r0 = R0;
            double r1 = R1 + u1 * R0;
            double r2 = R2 + 2.0 * u1 * R1 + u2 * R0;
            double r3 = R3 + 3.0 * u1 * R2 + 3.0 * u2 * R1 + u3 * R0;
            double r4 = R4 + 4.0 * u1 * R3 + 6.0 * u2 * R2 + 4.0 * u3 * R1 + u4 * R0;
            const double f = wyz * pre;
            r0 *= f;
            r1 *= f;
            r2 *= f;
            r3 *= f;
            r4 *= f;
            // sums over the row of t, t cx, t cy, t cz, ... with t = w G
            sm[0] += r0;
            sm[1] += r1;
            sm[2] += cy * r0;
            sm[3] += cz * r0;
            sm[4] += r2;
            sm[5] += cy * cy * r0;
            sm[6] += cz * cz * r0;
            sm[7] += cy * r1;
            sm[8] += cz * r1;
            sm[9] += cy * cz * r0;
            sm[10] += r3 + cyz2 * r1;             // cx |c|^2
            sm[11] += cy * (r2 + cyz2 * r0);      // cy |c|^2
            sm[12] += cz * (r2 + cyz2 * r0);      // cz |c|^2
            sm[13] += r4 + 2.0 * cyz2 * r2 + cyz2 * cyz2 * r0;  // |c|^4
        }
        // the 14 sums over the wave: the 16-value form of the sweep's moment
        // reduction (two slots unused), each sum then read from a lane that
        // holds it, so that every lane solves the same system
        double v16[16];
#pragma unroll
        for (int k = 0; k < 14; ++k) v16[k] = sm[k];
        v16[14] = v16[15] = 0.0;
        const double red = wave_reduce16(v16);
#pragma unroll
        for (int k = 0; k < 14; ++k) sm[k] = readlane_d(red, reduce16_lane(k));
        const double sc2 = sm[4] + sm[5] + sm[6];
        double A[5][5] = {{sm[0], sm[1], sm[2], sm[3], sc2},
                          {sm[1], sm[4], sm[7], sm[8], sm[10]},
                          {sm[2], sm[7], sm[5], sm[9], sm[11]},
                          {sm[3], sm[8], sm[9], sm[6], sm[12]},
                          {sc2, sm[10], sm[11], sm[12], sm[13]}};
        double bb[5] = {rho - sm[0], -sm[1], -sm[2], -sm[3], 1.5 * rho * T - sc2};
        if (!chol5_solve(A, bb, lam) && lane == 0) atomicOr(flag, 2);
    }
    if (lane == 0) {
        P[P_NU] = (S)nu;
        P[P_UX] = (S)Ux;
        P[P_UY] = (S)Uy;
        P[P_UZ] = (S)Uz;
        P[P_L0] = (S)(1.0 + lam[0]);
        P[P_L1] = (S)lam[1];
        P[P_L2] = (S)lam[2];
        P[P_L3] = (S)lam[3];
        P[P_L4] = (S)lam[4];
        P[P_QX] = (S)Axy;
        P[P_QY] = (S)Axz;
        P[P_QZ] = (S)Ayz;
        P[P_TWO_T] = (S)0;
    }
}

hipError_t launch_params_es(const Consts& C, const DevPtrs& D, const double* W, const double* stress,
                            const double* rho_w, void* params, void* etab, int prec, int* flag, hipStream_t st)
{
    if (prec == 0)
        params_es_kernel<double><<<C.N, 64, 0, st>>>(C, D, W, stress, rho_w, (double*)params, (double*)etab, flag);
    else
        params_es_kernel<float><<<C.N, 64, 0, st>>>(C, D, W, stress, rho_w, (float*)params, (float*)etab, flag);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Wall and free-stream emission shapes: the corrected equilibrium with unit
// density, velocity u_k, temperature T_k and no heat flux, over the whole
// velocity set, and its emitted-flux normaliser for every face orientation:
//   gout[k][s] = sum over xi.n > 0 of w (xi.n) ghat_k,  n the normal of side s
//   pointing into the gas (eq. "rho_wall" with the discrete quadrature).
// One block per kind.
// --------------------------------------------------------------------------

template <typename S>
__global__ __launch_bounds__(256) void emission_kernel(Consts C, DevPtrs D, const double* kind_state,
                                                       S* ghat, double* ghat64, double* gout)
{
    const int k = blockIdx.x;
    const double ux = kind_state[4 * k + 0], uy = kind_state[4 * k + 1], uz = kind_state[4 * k + 2];
    const double T = kind_state[4 * k + 3];
    __shared__ double lam_s[5];
    __shared__ double pre_s;
    __shared__ double red[6][256];
    if (threadIdx.x == 0) {
        const double pre = pow(M_PI * T, -1.5);
        double M[3][6];
        const double U3[3] = {ux, uy, uz};
        const int m3[3] = {C.mx, C.my, C.mz};
        for (int d = 0; d < 3; ++d) {
            for (int p = 0; p < 6; ++p) M[d][p] = 0.0;
            for (int a = 0; a < m3[d]; ++a) {
                const double c = D.xi[d * MAXM + a] - U3[d];
                double t = D.wt[d * MAXM + a] * exp(-c * c / T);
                for (int p = 0; p < 6; ++p) {
                    M[d][p] += t;
                    t *= c;
                }
            }
        }
        double lam[5] = {0, 0, 0, 0, 0};
        if (C.correct) correction_lambda(M[0], M[1], M[2], pre, 1.0, T, 0.0, 0, 0, 0, lam);
        for (int l = 0; l < 5; ++l) lam_s[l] = lam[l];
        pre_s = pre;
    }
    __syncthreads();
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int al = threadIdx.x; al < C.NV; al += blockDim.x) {
        const int a = al % C.mx, b = (al / C.mx) % C.my, c = al / (C.mx * C.my);
        const double xx = D.xi[a], xy = D.xi[MAXM + b], xz = D.xi[2 * MAXM + c];
        const double cx = xx - ux, cy = xy - uy, cz = xz - uz;
        const double c2 = cx * cx + cy * cy + cz * cz;
        const double fm = pre_s * exp(-c2 / T);
        const double g = fm * (1.0 + lam_s[0] + lam_s[1] * cx + lam_s[2] * cy + lam_s[3] * cz +
                               lam_s[4] * c2);
        ghat[(size_t)k * C.NV + al] = (S)g;
        ghat64[(size_t)k * C.NV + al] = g;
        const double w = D.wt[a] * D.wt[MAXM + b] * D.wt[2 * MAXM + c];
        const double xv[3] = {xx, xy, xz};
        for (int s = 0; s < 6; ++s) {
            const double xn = (s & 1) ? -xv[s >> 1] : xv[s >> 1];
            if (xn > 0) acc[s] += w * xn * g;
        }
    }
    for (int s = 0; s < 6; ++s) red[s][threadIdx.x] = acc[s];
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int s = 0; s < 6; ++s) red[s][threadIdx.x] += red[s][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 6) gout[k * 6 + threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_emission(const Consts& C, const DevPtrs& D, const double* kind_state, int nkind,
                           void* ghat, double* ghat64, double* gout, int prec, hipStream_t st)
{
    if (prec == 0)
        emission_kernel<double><<<nkind, 256, 0, st>>>(C, D, kind_state, (double*)ghat, ghat64, gout);
    else
        emission_kernel<float><<<nkind, 256, 0, st>>>(C, D, kind_state, (float*)ghat, ghat64, gout);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Initial wall densities: non-penetration flux of the initial corrected
// equilibrium at every wall face, divided by the emitted-flux normaliser.
// --------------------------------------------------------------------------

// initial wall densities: rho_w = (flux of the initial equilibrium into the
// wall) / (flux of the unit emission shape out of it).  One wave per cell;
// lanes stride over the velocities, then a shuffle tree (fixed order).
template <typename S>
__global__ __launch_bounds__(64) void wall_init_kernel(Consts C, DevPtrs D, const S* __restrict__ params,
                                                       const S* __restrict__ etab,
                                                       const double* __restrict__ gout,
                                                       double* __restrict__ rho_w)
{
    const int cell = blockIdx.x;
    const int lane = threadIdx.x;
    const uint32_t info = D.cellinfo[cell];
    if (lane < 6) rho_w[(size_t)lane * C.N + cell] = 0.0;
    if (info & SOLID_BIT) return;
    const S* P = params + (size_t)cell * PSTRIDE;
    const S* E = etab + (size_t)cell * C.MT;
    const double nu = (double)P[P_NU];
    const double Ux = (double)P[P_UX], Uy = (double)P[P_UY], Uz = (double)P[P_UZ];
    for (int s = 0; s < 6; ++s) {
        const uint32_t code = (info >> (4 * s)) & 15u;
        if (code == 0 || code == CODE_SPECULAR) continue;
        const int kind = (int)code - 1;
        if (!C.kind_wall[kind]) continue;
        const int d = s >> 1;
        double flux = 0.0;
        for (int v = lane; v < C.mx * C.my * C.mz; v += 64) {
            const int a = v % C.mx, b = (v / C.mx) % C.my, c = v / (C.mx * C.my);
            const double xv[3] = {D.xi[a], D.xi[MAXM + b], D.xi[2 * MAXM + c]};
            const double xn = (s & 1) ? -xv[d] : xv[d];  // xi . n, n into the gas
            if (!(xn < 0)) continue;
            const double cx = xv[0] - Ux, cy = xv[1] - Uy, cz = xv[2] - Uz;
            const double c2 = cx * cx + cy * cy + cz * cz;
            double poly = (double)P[P_L0] + (double)P[P_L1] * cx + (double)P[P_L2] * cy +
                          (double)P[P_L3] * cz + (double)P[P_L4] * c2;
            if (C.esbgk)
                poly *= exp(-((double)P[P_QX] * cx * cy + (double)P[P_QY] * cx * cz + (double)P[P_QZ] * cy * cz));
            else
                poly += ((double)P[P_QX] * cx + (double)P[P_QY] * cy + (double)P[P_QZ] * cz) *
                        (c2 * (double)P[P_TWO_T] - 5.0);
            const double nfs = (double)E[a] * (double)E[C.mx + b] * (double)E[C.mx + C.my + c] * poly;
            const double w = D.wt[a] * D.wt[MAXM + b] * D.wt[2 * MAXM + c];
            flux += w * (-xn) * nfs / nu;
        }
        for (int off = 32; off > 0; off >>= 1) flux += __shfl_xor(flux, off, 64);
        if (lane == 0) rho_w[(size_t)s * C.N + cell] = flux / gout[kind * 6 + s];
    }
}

hipError_t launch_wall_init(const Consts& C, const DevPtrs& D, const void* params, const void* etab,
                            const double* ghat64, const double* gout, double* rho_w, int prec,
                            hipStream_t st)
{
    (void)ghat64;
    if (prec == 0)
        wall_init_kernel<double><<<C.N, 64, 0, st>>>(C, D, (const double*)params, (const double*)etab, gout, rho_w);
    else
        wall_init_kernel<float><<<C.N, 64, 0, st>>>(C, D, (const float*)params, (const float*)etab, gout, rho_w);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Wave-level reduction of 13 FP64 values over the 64 lanes.
//
// Recursive halving: every step pairs two value registers and two lane
// groups, so the number of live registers halves while the lanes each
// register's partial spans double.  gfx950 permlane32/permlane16 swaps do the
// 32- and 16-lane steps, DPP row shifts with bank masks the 8- and 4-lane
// steps, quad permutes the last two.  After the call, lane
// L = 16 r + 4 b + x holds the full sum of value
//   idx(r, b) = {0, 8, 4, 12}[b] + {0, 2, 1, 3}[r]   (valid if <= 12).
// --------------------------------------------------------------------------

__device__ __forceinline__ void pl32_swap(double& x, double& y)
{
    // afterwards x = [x(0..31) | y(0..31)], y = [x(32..63) | y(32..63)]
    const unsigned x0 = (unsigned)__double2loint(x), x1 = (unsigned)__double2hiint(x);
    const unsigned y0 = (unsigned)__double2loint(y), y1 = (unsigned)__double2hiint(y);
    const auto r0 = __builtin_amdgcn_permlane32_swap(x0, y0, false, false);
    const auto r1 = __builtin_amdgcn_permlane32_swap(x1, y1, false, false);
    x = __hiloint2double((int)r1[0], (int)r0[0]);
    y = __hiloint2double((int)r1[1], (int)r0[1]);
}

__device__ __forceinline__ void pl16_swap(double& x, double& y)
{
    // rows of 16 lanes: afterwards x = [x r0, y r0, x r2, y r2], y = [x r1, y r1, x r3, y r3]
    const unsigned x0 = (unsigned)__double2loint(x), x1 = (unsigned)__double2hiint(x);
    const unsigned y0 = (unsigned)__double2loint(y), y1 = (unsigned)__double2hiint(y);
    const auto r0 = __builtin_amdgcn_permlane16_swap(x0, y0, false, false);
    const auto r1 = __builtin_amdgcn_permlane16_swap(x1, y1, false, false);
    x = __hiloint2double((int)r1[0], (int)r0[0]);
    y = __hiloint2double((int)r1[1], (int)r0[1]);
}

template <int CTRL, int ROWMASK, int BANKMASK>
__device__ __forceinline__ double dpp_merge(double old, double src)
{
    const int o0 = __double2loint(old), o1 = __double2hiint(old);
    const int s0 = __double2loint(src), s1 = __double2hiint(src);
    const int r0 = __builtin_amdgcn_update_dpp(o0, s0, CTRL, ROWMASK, BANKMASK, false);
    const int r1 = __builtin_amdgcn_update_dpp(o1, s1, CTRL, ROWMASK, BANKMASK, false);
    return __hiloint2double(r1, r0);
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double src)
{
    const int s0 = __double2loint(src), s1 = __double2hiint(src);
    const int r0 = __builtin_amdgcn_update_dpp(0, s0, CTRL, 0xF, 0xF, true);
    const int r1 = __builtin_amdgcn_update_dpp(0, s1, CTRL, 0xF, 0xF, true);
    return __hiloint2double(r1, r0);
}

constexpr int DPP_ROW_SHL8 = 0x108, DPP_ROW_SHR8 = 0x118;
constexpr int DPP_ROW_SHL4 = 0x104, DPP_ROW_SHR4 = 0x114;
constexpr int DPP_QUAD_2301 = 0x4E, DPP_QUAD_1032 = 0xB1;

__device__ __forceinline__ double halve8(double x, double y)
{
    // within each row: lanes 0-7 <- x(0..7) + x(8..15); lanes 8-15 <- y(0..7) + y(8..15)
    const double a = dpp_merge<DPP_ROW_SHR8, 0xF, 0xC>(x, y);  // lanes 8-15 take y(l-8)
    const double b = dpp_merge<DPP_ROW_SHL8, 0xF, 0x3>(y, x);  // lanes 0-7 take x(l+8)
    return a + b;
}

__device__ __forceinline__ double halve4(double x, double y)
{
    // banks of 4: bank0 <- x b0 + x b1, bank1 <- y b0 + y b1, bank2 <- x b2 + x b3, bank3 <- y b2 + y b3
    const double a = dpp_merge<DPP_ROW_SHR4, 0xF, 0xA>(x, y);
    const double b = dpp_merge<DPP_ROW_SHL4, 0xF, 0x5>(y, x);
    return a + b;
}

__device__ __forceinline__ double wave_reduce13(const double v[13])
{
    double r0 = v[0], r1 = v[1], r2 = v[2], r3 = v[3], r4 = v[4], r5 = v[5], r6 = v[6];
    double s0 = v[7], s1 = v[8], s2 = v[9], s3 = v[10], s4 = v[11], s5 = v[12], z = 0.0;
    // 64 -> 32 lanes: pairs (0,1) (2,3) (4,5) (6,7) (8,9) (10,11) (12,-)
    double a0 = r0, b0 = r1; pl32_swap(a0, b0); const double R0 = a0 + b0;
    double a1 = r2, b1 = r3; pl32_swap(a1, b1); const double R1 = a1 + b1;
    double a2 = r4, b2 = r5; pl32_swap(a2, b2); const double R2 = a2 + b2;
    double a3 = r6, b3 = s0; pl32_swap(a3, b3); const double R3 = a3 + b3;
    double a4 = s1, b4 = s2; pl32_swap(a4, b4); const double R4 = a4 + b4;
    double a5 = s3, b5 = s4; pl32_swap(a5, b5); const double R5 = a5 + b5;
    double a6 = s5, b6 = z;  pl32_swap(a6, b6); const double R6 = a6 + b6;
    // 32 -> 16 lanes
    double c0 = R0, d0 = R1; pl16_swap(c0, d0); const double Q0 = c0 + d0;  // rows: v0 v2 v1 v3
    double c1 = R2, d1 = R3; pl16_swap(c1, d1); const double Q1 = c1 + d1;  // rows: v4 v6 v5 v7
    double c2 = R4, d2 = R5; pl16_swap(c2, d2); const double Q2 = c2 + d2;  // rows: v8 v10 v9 v11
    double c3 = R6, d3 = z;  pl16_swap(c3, d3); const double Q3 = c3 + d3;  // rows: v12 - - -
    // 16 -> 8 -> 4 lanes within rows
    const double P0 = halve8(Q0, Q1);
    const double P1 = halve8(Q2, Q3);
    double O = halve4(P0, P1);  // banks: Q0 Q2 Q1 Q3
    // 4 -> 1
    O += dpp_mov<DPP_QUAD_2301>(O);
    O += dpp_mov<DPP_QUAD_1032>(O);
    return O;
}

// The same reduction of 16 values: the three slots that the 13-value form
// pads with zeros carry values 13..15 (one more 32-lane swap).  Lane
// L = 16 r + 4 b + x then holds the sum of value idx(r, b), all 16 valid.
__device__ __forceinline__ double wave_reduce16(const double v[16])
{
    double a0 = v[0], b0 = v[1]; pl32_swap(a0, b0); const double R0 = a0 + b0;
    double a1 = v[2], b1 = v[3]; pl32_swap(a1, b1); const double R1 = a1 + b1;
    double a2 = v[4], b2 = v[5]; pl32_swap(a2, b2); const double R2 = a2 + b2;
    double a3 = v[6], b3 = v[7]; pl32_swap(a3, b3); const double R3 = a3 + b3;
    double a4 = v[8], b4 = v[9]; pl32_swap(a4, b4); const double R4 = a4 + b4;
    double a5 = v[10], b5 = v[11]; pl32_swap(a5, b5); const double R5 = a5 + b5;
    double a6 = v[12], b6 = v[13]; pl32_swap(a6, b6); const double R6 = a6 + b6;
    double a7 = v[14], b7 = v[15]; pl32_swap(a7, b7); const double R7 = a7 + b7;
    double c0 = R0, d0 = R1; pl16_swap(c0, d0); const double Q0 = c0 + d0;
    double c1 = R2, d1 = R3; pl16_swap(c1, d1); const double Q1 = c1 + d1;
    double c2 = R4, d2 = R5; pl16_swap(c2, d2); const double Q2 = c2 + d2;
    double c3 = R6, d3 = R7; pl16_swap(c3, d3); const double Q3 = c3 + d3;  // rows: v12 v14 v13 v15
    const double P0 = halve8(Q0, Q1);
    const double P1 = halve8(Q2, Q3);
    double O = halve4(P0, P1);
    O += dpp_mov<DPP_QUAD_2301>(O);
    O += dpp_mov<DPP_QUAD_1032>(O);
    return O;
}

__device__ __forceinline__ int reduce13_index(int lane)
{
    const int r = lane >> 4, b = (lane >> 2) & 3;
    // base {0, 8, 4, 12}[b] = 4 * bitreverse2(b); row {0, 2, 1, 3}[r] = bitreverse2(r)
    const int rb = ((b & 1) << 1) | (b >> 1);
    const int rr = ((r & 1) << 1) | (r >> 1);
    return 4 * rb + rr;
}

__global__ __launch_bounds__(64) void selftest_reduce_kernel(const double* in, double* out)
{
    const int lane = threadIdx.x;
    double v[13];
    for (int k = 0; k < 13; ++k) v[k] = in[lane * 13 + k];
    const double s = wave_reduce13(v);
    const int idx = reduce13_index(lane);
    if ((lane & 3) == 0 && idx < 13) out[idx] = s;
}

hipError_t launch_selftest_reduce(const double* in, double* out, hipStream_t st)
{
    selftest_reduce_kernel<<<1, 64, 0, st>>>(in, out);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// A3/A4: the sweep.
//
// Work unit = (octant o, brick (I,J,K) in the octant's sweep-reflected
// coordinates, tile of 64 lanes).  Each lane owns VL discrete velocities of
// the octant that share (xi_y, xi_z) and march through the brick in upwind
// order: z planes outer, y rows, x cells inner.  The brick's current plane of
// f lives in registers (plane[v][jj][ii] holds the newest value of that
// column), so in-brick upwind operands never leave the VGPRs; only the three
// inflow faces are read from, and the three outflow faces written to, HBM
// face buffers (double-buffered by brick parity along each axis).  All bricks
// of one diagonal I+J+K = T are independent and form one launch; the
// per-velocity upwind system is triangular, so any such order reproduces the
// sequential sweep exactly.
//
// Per cell the lane evaluates nu * f~S from the cell's FP64-derived
// parameters (wave-uniform, scalar loads) and the separable Gaussian tables,
// updates f, and accumulates the 13 raw moments of its velocities; one
// wave reduction per cell gives the tile's partial, written to a
// deterministic slot partial[o*ntiles + tile][cell].
// --------------------------------------------------------------------------

// byte-offset load/store: a wave-uniform base pointer plus a 32-bit per-lane
// byte offset, so that the address is one SGPR pair plus one VGPR
template <typename T>
__device__ __forceinline__ T ldb(const T* base, unsigned off)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ void stb(T* base, unsigned off, T v)
{
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off) = v;
}
// gather through a raw buffer resource made from the (wave-uniform) base:
// the resource in SGPRs plus the 32-bit lane offset, no per-lane 64-bit
// address arithmetic (a plain load adds the lane offset, held as a 64-bit
// register pair, to the base for every gather)
template <typename T>
__device__ __forceinline__ T ldg(const T* base, unsigned off)
{
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, -1, 0x00020000);
    T v;
    if constexpr (sizeof(T) == 8) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
        __builtin_memcpy(&v, &w, 8);
    } else {
        const auto w = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
        __builtin_memcpy(&v, &w, 4);
    }
    return v;
}
// wait until no vector-memory load or store of this wave is outstanding,
// leaving the other counters alone: s_waitcnt with vmcnt 0 (bits 3:0 and
// 15:14), expcnt 7 (bits 6:4) and lgkmcnt 15 (bits 11:8), i.e. no wait on
// those two (gfx9 encoding)
__device__ __forceinline__ void wait_vector_memory()
{
    __builtin_amdgcn_s_waitcnt(0x0F70);
}
// an empty statement that reads x: x stays in its register up to here
template <typename T>
__device__ __forceinline__ void keep_alive(T x)
{
    asm volatile("" ::"v"(x));
}
// streaming store (non-temporal hint): the outflow faces and moment partials
// are read back only by a later launch, so they should not displace the cell
// tables and faces of the running launch from the caches
template <typename T>
__device__ __forceinline__ void stb_nt(T* base, unsigned off, T v)
{
    __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off));
}

// The VL values of a lane in a face row: row at byte offset cofs (uniform)
// from the face base, the lane's values at lofs within it.  COH: loads and
// stores coherent at device scope -- buffer instructions with the sc1 bit
// (the lane offset in a VGPR, the row offset in an SGPR), which bypass the
// per-CU caches and the per-XCD L2 whose copies of a face row are not kept
// coherent while one kernel runs -- for faces that a later brick of the
// same launch reads.  Otherwise plain loads and streaming stores (the
// reader is a later launch).
constexpr int BUF_SC1 = 16;                       // cache-policy bit: device scope
constexpr int BUF_WORD3 = 0x00020000;             // gfx9 raw buffer: 32-bit data format
template <typename S>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t face_rsrc(const S* base)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<S*>(base), (short)0, -1, BUF_WORD3);
}
template <bool COH, typename S, int VL>
__device__ __forceinline__ void load_face(const S* base, unsigned cofs, unsigned lofs, S (&out)[VL])
{
    if constexpr (!COH) {
        const S* src = reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + cofs);
#pragma unroll
        for (int v = 0; v < VL; ++v) out[v] = ldb(src, lofs + v * (unsigned)sizeof(S));
    } else {
        constexpr int NB = VL * (int)sizeof(S);
        static_assert(NB % 4 == 0, "face values are whole dwords");
        const __amdgpu_buffer_rsrc_t r = face_rsrc(base);
        unsigned w[NB / 4];
        int at = 0;
#pragma unroll
        for (; at + 16 <= NB; at += 16) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, lofs + at, cofs, BUF_SC1);
            w[at / 4] = x[0]; w[at / 4 + 1] = x[1]; w[at / 4 + 2] = x[2]; w[at / 4 + 3] = x[3];
        }
        if constexpr (NB % 16 >= 8) {
            const auto x = __builtin_amdgcn_raw_buffer_load_b64(r, lofs + (NB / 16) * 16, cofs, BUF_SC1);
            w[(NB / 16) * 4] = x[0]; w[(NB / 16) * 4 + 1] = x[1];
        }
        if constexpr (NB % 8 == 4)
            w[NB / 4 - 1] = __builtin_amdgcn_raw_buffer_load_b32(r, lofs + NB - 4, cofs, BUF_SC1);
#pragma unroll
        for (int v = 0; v < VL; ++v) {
            if constexpr (sizeof(S) == 8)
                out[v] = __builtin_bit_cast(S, (unsigned long long)w[2 * v] | ((unsigned long long)w[2 * v + 1] << 32));
            else
                out[v] = __builtin_bit_cast(S, w[v]);
        }
    }
}
template <bool COH, typename S, int VL>
__device__ __forceinline__ void store_face(S* base, unsigned cofs, unsigned lofs, const S (&val)[VL])
{
    if constexpr (!COH) {
        S* dst = reinterpret_cast<S*>(reinterpret_cast<char*>(base) + cofs);
#pragma unroll
        for (int v = 0; v < VL; ++v) stb_nt(dst, lofs + v * (unsigned)sizeof(S), val[v]);
    } else {
        constexpr int NB = VL * (int)sizeof(S);
        const __amdgpu_buffer_rsrc_t r = face_rsrc(base);
        unsigned w[NB / 4];
#pragma unroll
        for (int v = 0; v < VL; ++v) {
            if constexpr (sizeof(S) == 8) {
                const unsigned long long u = __builtin_bit_cast(unsigned long long, val[v]);
                w[2 * v] = (unsigned)u;
                w[2 * v + 1] = (unsigned)(u >> 32);
            } else {
                w[v] = __builtin_bit_cast(unsigned, val[v]);
            }
        }
        using u4 = __attribute__((ext_vector_type(4))) unsigned;
        using u2 = __attribute__((ext_vector_type(2))) unsigned;
        int at = 0;
#pragma unroll
        for (; at + 16 <= NB; at += 16) {
            const u4 x = {w[at / 4], w[at / 4 + 1], w[at / 4 + 2], w[at / 4 + 3]};
            __builtin_amdgcn_raw_buffer_store_b128(x, r, lofs + at, cofs, BUF_SC1);
        }
        if constexpr (NB % 16 >= 8) {
            const u2 x = {w[(NB / 16) * 4], w[(NB / 16) * 4 + 1]};
            __builtin_amdgcn_raw_buffer_store_b64(x, r, lofs + (NB / 16) * 16, cofs, BUF_SC1);
        }
        if constexpr (NB % 8 == 4) __builtin_amdgcn_raw_buffer_store_b32(w[NB / 4 - 1], r, lofs + NB - 4, cofs, BUF_SC1);
    }
}

// O2: second-order upwind.  Each face carries the upwind cell's value
// extrapolated linearly from that cell and its own upwind neighbour,
// F = f + (f - f_up)/2 (F = f when that cell's upwind side is a boundary);
// per axis the cell balance a (F_out - F_in) makes the unknown enter with
// 3a/2 behind an interior face (a behind a boundary) and takes F_in + f_up/2
// from the upwind side.  Carried along: x -- the previous cell's (f, F) in
// registers; y -- f of the two previous rows from the plane, F rebuilt from
// them (a bit per plane cell records a boundary behind it); z -- a second
// LDS plane with each column's newest F.  Faces and the mirror plane hold
// (f, F) pairs; a symmetry plane is an interior face (the mirror image is
// the cell beyond it).  Three more raw moments, sum w xi_d (F_d - f), turn
// the cell-value fluxes into face fluxes for the wall densities.
// ES: the ES-BGK Gaussian in place of the Shakhov polynomial: no heat-flux
// term, and the per-point cross factor exp(-(cx B + C)) of the anisotropic
// Gaussian, B = A_xy cy + A_xz cz and C = A_yz cy cz fixed per lane and cell.
// ES-BGK: the cross factor exp(-(c_x B + C)) of each of a lane's velocities.
// With REC (a uniform x axis) the lane's nodes lie one step apart, or repeat
// the last node of the half axis in its unused slots, so each factor follows
// from the one before by one product with exp(-step B): two exponentials per
// lane and cell instead of one per velocity (taken where an exponential costs
// many instructions, in FP64); otherwise one exponential per velocity.
template <typename T>
__device__ __forceinline__ T es_exp(T a)
{
    if constexpr (sizeof(T) == 8)
        return exp(a);
    else
        return __expf(a);
}

template <typename T, bool REC>
struct EsCross {
    T cur, step;
    __device__ __forceinline__ EsCross(T x0, T x1, T Ux, T B, T Cc) : cur(0), step(0)
    {
        if constexpr (REC) {
            cur = es_exp(-((x0 - Ux) * B + Cc));
            step = es_exp(-(x1 - x0) * B);
        }
    }
    // the factor of velocity v (called for v = 0, 1, ... in order)
    __device__ __forceinline__ T at(int v, T xv, T xprev, T cx, T B, T Cc)
    {
        if constexpr (REC) {
            if (v > 0 && xv != xprev) cur *= step;
            return cur;
        } else {
            return es_exp(-(cx * B + Cc));
        }
    }
};

template <typename S, int VL, int BX, int BY, bool NU, bool O2 = false, bool ES = false>
__device__ __forceinline__ void sweep_body(const SweepArgs<S>& A, const S* __restrict__ params,
                                           const S* __restrict__ etab, const S* __restrict__ ghat,
                                           const double* __restrict__ lanetab, const int* __restrict__ bricks,
                                           S* __restrict__ xface, S* __restrict__ yface, S* __restrict__ zface,
                                           S* __restrict__ spec, double* __restrict__ partial, S* __restrict__ plane)
{
    const int lane = threadIdx.x;
    int bid = blockIdx.x;
    // XCD-aware order: consecutive block ids go round-robin over the 8 XCDs,
    // so regroup them to give each XCD a contiguous range of work units
    // (neighbouring tiles of the same brick share the cell tables in L2).
    {
        const int nb = A.nblocks;
        const int per = nb / 8, rem = nb % 8;
        const int xcd = bid % 8, k = bid / 8;
        const int start = xcd * per + (xcd < rem ? xcd : rem);
        bid = start + k;
    }
    const int tile = bid % A.ntiles;
    bid /= A.ntiles;
    const int bi = bid % A.brick_cnt;
    const int o = A.oct_base + bid / A.brick_cnt;
    const int I = bricks[4 * (A.brick_off + bi) + 0];
    const int J = bricks[4 * (A.brick_off + bi) + 1];
    const int K = bricks[4 * (A.brick_off + bi) + 2];
    const bool px = (o & 1) != 0, py = (o & 2) != 0, pz = (o & 4) != 0;
    const int slot = tile * 64 + lane;
    const int nx = A.nx, ny = A.ny, nz = A.nz, MT = A.MT;
    constexpr unsigned SB = sizeof(S);
    const size_t fstride = (size_t)A.slots * VL;
    const unsigned lofs = (unsigned)slot * VL * SB;

    const int iend = min(BX, nx - I * BX), jend = min(BY, ny - J * BY);
    const int kend = min(A.bz, nz - K * A.bz);
    const bool wx = I < A.nbx - 1, wy = J < A.nby - 1, wz = K < A.nbz - 1;
    const int ir0 = I * BX, jr0 = J * BY, kr0 = K * A.bz;
    // cell index steps along the octant's sweep directions
    const int si = px ? 1 : -1, sj = py ? nx : -nx, sk = pz ? nx * ny : -nx * ny;
    const int cell0 = (px ? ir0 : nx - 1 - ir0) + nx * ((py ? jr0 : ny - 1 - jr0) + ny * (pz ? kr0 : nz - 1 - kr0));

    // face rows: (x) one slot row per (kr, jr), (y) per (kr, ir), (z) per (jr, ir)
    const S* xin = xface + ((size_t)(o * 2 + ((I - 1) & 1)) * nz * ny + (size_t)kr0 * ny + jr0) * fstride;
    S* xout = xface + ((size_t)(o * 2 + (I & 1)) * nz * ny + (size_t)kr0 * ny + jr0) * fstride;
    const S* yin = yface + ((size_t)(o * 2 + ((J - 1) & 1)) * nz * nx + (size_t)kr0 * nx + ir0) * fstride;
    S* yout = yface + ((size_t)(o * 2 + (J & 1)) * nz * nx + (size_t)kr0 * nx + ir0) * fstride;
    const S* zin = zface + ((size_t)(o * 2 + ((K - 1) & 1)) * ny * nx + (size_t)jr0 * nx + ir0) * fstride;
    S* zout = zface + ((size_t)(o * 2 + (K & 1)) * ny * nx + (size_t)jr0 * nx + ir0) * fstride;
    S* sbuf = A.spec_on ? spec + (size_t)(o & 3) * ny * nx * fstride : nullptr;
    // second order: the F layers of the same faces and mirror plane
    const S* xgin = nullptr; S* xgout = nullptr;
    const S* ygin = nullptr; S* ygout = nullptr;
    const S* zgin = nullptr; S* zgout = nullptr;
    S* sgbuf = nullptr;
    if constexpr (O2) {
        xgin = A.xgface + (xin - xface);
        xgout = A.xgface + (xout - xface);
        ygin = A.ygface + (yin - yface);
        ygout = A.ygface + (yout - yface);
        zgin = A.zgface + (zin - zface);
        zgout = A.zgface + (zout - zface);
        sgbuf = A.spec_on ? A.specg + (size_t)(o & 3) * ny * nx * fstride : nullptr;
    }

    // the brick's newest plane of f: lds(jj, ii, v) = plane[((jj*BX + ii)*VL + v)*64 + lane];
    // second order: ldz, the newest F along z of each column, follows it
    auto lds = [&](int jj, int ii, int v) -> S& { return plane[((jj * BX + ii) * VL + v) * 64 + lane]; };
    auto ldz = [&](int jj, int ii, int v) -> S& {
        return plane[((BY * BX + jj * BX + ii) * VL + v) * 64 + lane];
    };

    // ---- lane constants
    const double* lt = lanetab + ((size_t)o * A.slots + slot) * A.lstride;
    const double xiy_d = lt[0], xiz_d = lt[1];
    const S xiy = (S)xiy_d, xiz = (S)xiz_d;
    const S ay = (S)lt[2], az = (S)lt[3];
    const int vb = (int)lt[4], vc = (int)lt[5];
    // |xi_x| / h_x is formed per cell from the node and a wave-uniform
    // factor (the octant's sign over h_x, or the sign alone on a non-uniform
    // mesh, whose cells bring their own inverse size): fewer live registers
    S xix[VL];
    double wm0[VL], wm1[VL], wm2[VL], wm3[VL];
    unsigned oa[VL], oal[VL];
#pragma unroll
    for (int v = 0; v < VL; ++v) {
        const double x = lt[LT_SHARED + LT_PER_V * v + 0];
        const double w = lt[LT_SHARED + LT_PER_V * v + 2];
        const int a = (int)lt[LT_SHARED + LT_PER_V * v + 3];
        xix[v] = (S)x;
        oa[v] = (unsigned)a * SB;
        oal[v] = (unsigned)(a + A.mx * (vb + A.my * vc)) * SB;
        wm0[v] = w;
        wm1[v] = w * x;
        wm2[v] = w * x * x;
        wm3[v] = w * x * x * x;
    }
    const unsigned ob = (unsigned)(A.mx + vb) * SB, oc = (unsigned)(A.mx + A.my + vc) * SB;
    const S sgx = px ? (S)A.rdx : -(S)A.rdx;
    const double yz2 = xiy_d * xiy_d + xiz_d * xiz_d;
    const double xiyy = xiy_d * xiy_d, xizz = xiz_d * xiz_d, xiyz = xiy_d * xiz_d;
    const int sideX = px ? 0 : 1, sideY = py ? 2 : 3, sideZ = pz ? 4 : 5;
    const int shX = 4 * sideX, shY = 4 * sideY, shZ = 4 * sideZ;
    const int ridx = reduce13_index(lane);
    const bool writer = (lane & 3) == 0;  // one lane per slot 0..15 of the record
    const unsigned oridx = (unsigned)ridx * 8u;
    double* part = partial + ((size_t)(o * A.ntiles + tile) * A.N) * PREC;

    for (int kk = 0; kk < kend; ++kk) {
        const int kcell = cell0 + kk * sk;
        uint32_t ybnd = 0;  // second order: plane cells whose y upwind side is a boundary
        for (int jj = 0; jj < jend; ++jj) {
            const int rcell = kcell + jj * sj;
            const S* xrow_in = xin + ((size_t)kk * ny + jj) * fstride;
            S* xrow_out = xout + ((size_t)kk * ny + jj) * fstride;
            S prev[VL];
            S prevF[VL];  // second order: the previous cell's F along x
            for (int ii = 0; ii < iend; ++ii) {
                const int cell = rcell + ii * si;
                const S* P = params + (size_t)cell * PSTRIDE;
                const uint32_t info = reinterpret_cast<const uint32_t*>(P + P_INFO)[0];
                if (info & SOLID_BIT) continue;
                const S* E = etab + (size_t)cell * MT;

                // ---- upwind operands: 0 = interior neighbour (in the plane,
                //      the previous cell, or the upwind brick's face), 8 =
                //      symmetry plane, 7 = solid body, else the box face
                // second order: fx.. hold F_in + f_up / 2 behind an interior
                // face, ux.. hold f_up, and ix.. say which faces are interior
                S fx[VL], fy[VL], fz[VL];
                S ux[VL], uy[VL], uz[VL];
                bool ixf = false, iyf = false, izf = false;
                {
                    const uint32_t code = (info >> shX) & 15u;
                    if (code == 0) {
                        if constexpr (O2) {
                            ixf = true;
                            if (ii > 0) {
#pragma unroll
                                for (int v = 0; v < VL; ++v) {
                                    ux[v] = prev[v];
                                    fx[v] = prevF[v] + (S)0.5 * prev[v];
                                }
                            } else {
                                const S* grow_in = xgin + ((size_t)kk * ny + jj) * fstride;
#pragma unroll
                                for (int v = 0; v < VL; ++v) {
                                    ux[v] = ldb(xrow_in, lofs + v * SB);
                                    fx[v] = ldb(grow_in, lofs + v * SB) + (S)0.5 * ux[v];
                                }
                            }
                        } else if (ii > 0) {
#pragma unroll
                            for (int v = 0; v < VL; ++v) fx[v] = prev[v];
                        } else {
#pragma unroll
                            for (int v = 0; v < VL; ++v) fx[v] = ldb(xrow_in, lofs + v * SB);
                        }
                    } else {
                        const S rf = P[P_RHO_SIDE + sideX];
                        const S* g = ghat + (size_t)(code - 1) * A.NV;
#pragma unroll
                        for (int v = 0; v < VL; ++v) fx[v] = rf * ldb(g, oal[v]);
                    }
                }
                {
                    const uint32_t code = (info >> shY) & 15u;
                    if constexpr (O2) {
                        if (code != 0) ybnd |= 1u << (jj * BX + ii);
                    }
                    if (code == 0) {
                        if constexpr (O2) {
                            iyf = true;
                            if (jj > 0) {
                                // F of the row behind: from its own upwind row
                                const bool edge = (ybnd >> ((jj - 1) * BX + ii)) & 1u;
                                const S* f2row = yin + ((size_t)kk * nx + ii) * fstride;
#pragma unroll
                                for (int v = 0; v < VL; ++v) {
                                    const S fu = lds(jj - 1, ii, v);
                                    S Fu = fu;
                                    if (!edge) {
                                        const S f2 = jj >= 2 ? lds(jj - 2, ii, v) : ldb(f2row, lofs + v * SB);
                                        Fu = (S)1.5 * fu - (S)0.5 * f2;
                                    }
                                    uy[v] = fu;
                                    fy[v] = Fu + (S)0.5 * fu;
                                }
                            } else {
                                const S* src = yin + ((size_t)kk * nx + ii) * fstride;
                                const S* gsrc = ygin + ((size_t)kk * nx + ii) * fstride;
#pragma unroll
                                for (int v = 0; v < VL; ++v) {
                                    uy[v] = ldb(src, lofs + v * SB);
                                    fy[v] = ldb(gsrc, lofs + v * SB) + (S)0.5 * uy[v];
                                }
                            }
                        } else if (jj > 0) {
#pragma unroll
                            for (int v = 0; v < VL; ++v) fy[v] = lds(jj - 1, ii, v);
                        } else {
                            const S* src = yin + ((size_t)kk * nx + ii) * fstride;
#pragma unroll
                            for (int v = 0; v < VL; ++v) fy[v] = ldb(src, lofs + v * SB);
                        }
                    } else {
                        const S rf = P[P_RHO_SIDE + sideY];
                        const S* g = ghat + (size_t)(code - 1) * A.NV;
#pragma unroll
                        for (int v = 0; v < VL; ++v) fy[v] = rf * ldb(g, oal[v]);
                    }
                }
                {
                    const uint32_t code = (info >> shZ) & 15u;
                    if (O2 && (code == 0 || code == CODE_SPECULAR)) {
                        izf = true;
                        if (code == 0 && kk > 0) {
#pragma unroll
                            for (int v = 0; v < VL; ++v) {
                                uz[v] = lds(jj, ii, v);
                                fz[v] = ldz(jj, ii, v) + (S)0.5 * uz[v];
                            }
                        } else {
                            // the upwind brick's face, or the mirror image
                            // beyond the symmetry plane
                            const S* src;
                            const S* gsrc;
                            if (code == 0) {
                                src = zin + ((size_t)jj * nx + ii) * fstride;
                                gsrc = zgin + ((size_t)jj * nx + ii) * fstride;
                            } else {
                                const int i = px ? ir0 + ii : nx - 1 - (ir0 + ii);
                                const int j = py ? jr0 + jj : ny - 1 - (jr0 + jj);
                                src = sbuf + ((size_t)j * nx + i) * fstride;
                                gsrc = sgbuf + ((size_t)j * nx + i) * fstride;
                            }
#pragma unroll
                            for (int v = 0; v < VL; ++v) {
                                uz[v] = ldb(src, lofs + v * SB);
                                fz[v] = ldb(gsrc, lofs + v * SB) + (S)0.5 * uz[v];
                            }
                        }
                    } else if (code == 0) {
                        if (kk > 0) {
#pragma unroll
                            for (int v = 0; v < VL; ++v) fz[v] = lds(jj, ii, v);
                        } else {
                            const S* src = zin + ((size_t)jj * nx + ii) * fstride;
#pragma unroll
                            for (int v = 0; v < VL; ++v) fz[v] = ldb(src, lofs + v * SB);
                        }
                    } else if (code == CODE_SPECULAR) {
                        // inflow of a +z velocity at z = 0: the outflow of its
                        // mirror image (same lane, same octant-local index)
                        const int i = px ? ir0 + ii : nx - 1 - (ir0 + ii);
                        const int j = py ? jr0 + jj : ny - 1 - (jr0 + jj);
                        const S* src = sbuf + ((size_t)j * nx + i) * fstride;
#pragma unroll
                        for (int v = 0; v < VL; ++v) fz[v] = ldb(src, lofs + v * SB);
                    } else {
                        const S rf = P[P_RHO_SIDE + sideZ];
                        const S* g = ghat + (size_t)(code - 1) * A.NV;
#pragma unroll
                        for (int v = 0; v < VL; ++v) fz[v] = rf * ldb(g, oal[v]);
                    }
                }

                // ---- equilibrium (wave-uniform cell parameters) and update
                const S nu = P[P_NU], Ux = P[P_UX], Uy = P[P_UY], Uz = P[P_UZ];
                const S L0 = P[P_L0], L1 = P[P_L1], L2 = P[P_L2], L3 = P[P_L3], L4 = P[P_L4];
                const S qx = P[P_QX], qy = P[P_QY], qz = P[P_QZ], tT = P[P_TWO_T];
                const S gyz = ldb(E, ob) * ldb(E, oc);
                const S cy = xiy - Uy, cz = xiz - Uz;
                const S cyz2 = cy * cy + cz * cz;
                const S Lyz = L0 + L2 * cy + L3 * cz;
                const S Qyz = qy * cy + qz * cz;
                // ES-BGK: qx, qy, qz hold A_xy, A_xz, A_yz
                const S Bes = qx * cy + qy * cz, Ces = qz * cy * cz;
                EsCross<S, false> cross(xix[0], xix[0], Ux, Bes, Ces);
                // upwind coefficients: lane constants |xi_d| / h_d (uniform mesh),
                // or |xi_d| times the cell's inverse sizes (non-uniform mesh)
                S ayc = ay, azc = az, sx = sgx;
                if constexpr (NU) {
                    sx = sgx * P[P_IDX];
                    ayc = ay * P[P_IDY];
                    azc = az * P[P_IDZ];
                }
                const S aynu = ayc + azc + nu;
                double u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
                double e0 = 0.0, e1 = 0.0, e2 = 0.0;  // second order: sum w (F_d - f)
                S Fy[VL], Fz[VL];
                // second order: 3a/2 behind an interior face
                const S kx = O2 && ixf ? (S)1.5 : (S)1, ky = O2 && iyf ? (S)1.5 : (S)1;
                const S kz = O2 && izf ? (S)1.5 : (S)1;
                const S ayk = ayc * ky, azk = azc * kz;
#pragma unroll
                for (int v = 0; v < VL; ++v) {
                    const S cx = xix[v] - Ux;
                    const S c2 = cx * cx + cyz2;
                    S nfs;
                    if constexpr (ES) {
                        const S poly = Lyz + L1 * cx + L4 * c2;
                        nfs = gyz * ldb(E, oa[v]) * poly * cross.at(v, xix[v], xix[v > 0 ? v - 1 : 0], cx, Bes, Ces);
                    } else {
                        const S poly = Lyz + L1 * cx + L4 * c2 + (Qyz + qx * cx) * (c2 * tT - (S)5);
                        nfs = gyz * ldb(E, oa[v]) * poly;
                    }
                    const S axv = xix[v] * sx;
                    S f;
                    if constexpr (O2) {
                        const S axk = axv * kx;
                        const S num = axv * fx[v] + ayc * fy[v] + azc * fz[v] + nfs;
                        f = num * fast_rcp(axk + ayk + azk + nu);
                        // what this cell carries through its downstream faces
                        const S dx = ixf ? (S)0.5 * (f - ux[v]) : (S)0;
                        const S dy = iyf ? (S)0.5 * (f - uy[v]) : (S)0;
                        const S dz = izf ? (S)0.5 * (f - uz[v]) : (S)0;
                        prevF[v] = f + dx;
                        Fy[v] = f + dy;
                        Fz[v] = f + dz;
                        ldz(jj, ii, v) = Fz[v];
                        e0 += wm1[v] * (double)dx;
                        e1 += wm0[v] * (double)dy;
                        e2 += wm0[v] * (double)dz;
                    } else {
                        const S num = axv * fx[v] + ayc * fy[v] + azc * fz[v] + nfs;
                        f = num * fast_rcp(axv + aynu);
                    }
                    prev[v] = f;
                    lds(jj, ii, v) = f;
                    const double fd = (double)f;
                    u0 += wm0[v] * fd;
                    u1 += wm1[v] * fd;
                    u2 += wm2[v] * fd;
                    u3 += wm3[v] * fd;
                }

                // ---- outflow faces for the downstream bricks
                if (ii == BX - 1 && wx) {
#pragma unroll
                    for (int v = 0; v < VL; ++v) stb_nt(xrow_out, lofs + v * SB, prev[v]);
                    if constexpr (O2) {
                        S* g = xgout + ((size_t)kk * ny + jj) * fstride;
#pragma unroll
                        for (int v = 0; v < VL; ++v) stb_nt(g, lofs + v * SB, prevF[v]);
                    }
                }
                if (jj == BY - 1 && wy) {
#pragma unroll
                    for (int v = 0; v < VL; ++v) stb_nt(yout + ((size_t)kk * nx + ii) * fstride, lofs + v * SB, prev[v]);
                    if constexpr (O2) {
#pragma unroll
                        for (int v = 0; v < VL; ++v)
                            stb_nt(ygout + ((size_t)kk * nx + ii) * fstride, lofs + v * SB, Fy[v]);
                    }
                }
                if (kk == A.bz - 1 && wz) {
#pragma unroll
                    for (int v = 0; v < VL; ++v) stb_nt(zout + ((size_t)jj * nx + ii) * fstride, lofs + v * SB, prev[v]);
                    if constexpr (O2) {
#pragma unroll
                        for (int v = 0; v < VL; ++v)
                            stb_nt(zgout + ((size_t)jj * nx + ii) * fstride, lofs + v * SB, Fz[v]);
                    }
                }
                if (sbuf != nullptr && !pz && kr0 + kk == nz - 1) {
                    const int i = px ? ir0 + ii : nx - 1 - (ir0 + ii);
                    const int j = py ? jr0 + jj : ny - 1 - (jr0 + jj);
                    S* dst = sbuf + ((size_t)j * nx + i) * fstride;
#pragma unroll
                    for (int v = 0; v < VL; ++v) stb_nt(dst, lofs + v * SB, prev[v]);
                    if constexpr (O2) {
                        S* g = sgbuf + ((size_t)j * nx + i) * fstride;
#pragma unroll
                        for (int v = 0; v < VL; ++v) stb_nt(g, lofs + v * SB, Fz[v]);
                    }
                }

                // ---- 13 raw moments of this tile at this cell
                double m[O2 ? 16 : 13];
                m[0] = u0;
                m[1] = u1;
                m[2] = xiy_d * u0;
                m[3] = xiz_d * u0;
                m[4] = u2;
                m[5] = xiyy * u0;
                m[6] = xizz * u0;
                m[7] = xiy_d * u1;
                m[8] = xiz_d * u1;
                m[9] = xiyz * u0;
                m[10] = u3 + yz2 * u1;
                const double t2 = u2 + yz2 * u0;
                m[11] = xiy_d * t2;
                m[12] = xiz_d * t2;
                double tot;
                if constexpr (O2) {
                    m[13] = e0;
                    m[14] = xiy_d * e1;
                    m[15] = xiz_d * e2;
                    tot = wave_reduce16(m);
                } else {
                    tot = wave_reduce13(m);
                }
                if (writer) stb_nt(part + (size_t)cell * PREC, oridx, tot);
            }
        }
    }
}

// the LDS plane of the block's wave (dynamic size)
extern __shared__ __align__(16) unsigned char dvm_sweep_lds[];

// Software-pipelined form of the same sweep.  The cells of the brick are
// visited in the same order through one flat loop; while cell n is computed,
// the loads of cell n+1 are already in flight: its Gaussian-table gathers and,
// by position alone, the inflow values it will take from the upwind bricks'
// x and y faces (when its own boundary code says otherwise, e.g. next to a
// solid, the prefetched value is simply not used).  The first plane's z inflow
// is staged into the LDS plane before the loop, so every plane takes its z
// upwind operand from LDS.  Moments are accumulated from the node weight and
// abscissa (three more multiplies per velocity instead of four per-velocity
// weight products held in registers).
// O2 / ES: the second-order sweep and the ES-BGK Gaussian, as in the plain
// body; with O2 the (f, F) pairs of the faces are prefetched together, the
// first plane's F along z is staged into the second LDS plane with its f,
// and the row-behind-the-face f that rebuilds F along y is prefetched for
// the second row.
// The work unit of a block of a per-diagonal launch: block ids are
// regrouped so that each XCD gets a contiguous range of (brick, tile) units.
struct WorkUnit {
    int o, tile, I, J, K;
};
template <typename S>
__device__ __forceinline__ WorkUnit diagonal_unit(const SweepArgs<S>& A, const int* __restrict__ bricks)
{
    int bid = blockIdx.x;
    {
        const int nb = A.nblocks;
        const int per = nb / 8, rem = nb % 8;
        const int xcd = bid % 8, k = bid / 8;
        const int start = xcd * per + (xcd < rem ? xcd : rem);
        bid = start + k;
    }
    WorkUnit u;
    u.tile = bid % A.ntiles;
    bid /= A.ntiles;
    const int bi = bid % A.brick_cnt;
    u.o = A.oct_base + bid / A.brick_cnt;
    u.I = bricks[4 * (A.brick_off + bi) + 0];
    u.J = bricks[4 * (A.brick_off + bi) + 1];
    u.K = bricks[4 * (A.brick_off + bi) + 2];
    return u;
}

// Cells of the pipelined body's brick plane whose z inflow stays in
// registers: an FP64 plane of 4 x 2 cells with 4 velocities per lane takes
// 16 KB of LDS per wave, which leaves 2.5 waves per SIMD where the registers
// allow 3; holding the last row's last two cells (16 VGPRs) brings it to
// 12 KB.  The same for the second-order FP64 form with 2 per lane, whose f
// and F planes take 16 KB together (its two cells' f and F: 16 VGPRs).
// Those cells are only ever read for their own z inflow (the row behind a
// cell is the row before it, and the faces are stored from the registers
// of the cell just computed).  Shakhov's model only: the ES-BGK form would
// pass 168 VGPRs (2 waves per SIMD); not in the dependency-driven form,
// whose registers are full.
template <typename S, int VL, int BX, int BY, bool O2, bool ES, bool COH>
__host__ __device__ constexpr int zreg_cells()
{
    return (!ES && !COH && sizeof(S) == 8 && BX == 4 && BY == 2 && (O2 ? VL == 2 : VL == 4)) ? 2 : 0;
}

// PT: type of the per-cell parameter record, the Gaussian factor tables and
// the equilibrium evaluation (S, or double beside FP32 storage of f: the
// equilibrium then enters the FP32 update rounded once).
// XU: the x velocity axis is uniform (ES-BGK takes its cross factors by
// recurrence along the lane's nodes).
template <typename S, int VL, int BX, int BY, bool NU, bool O2 = false, bool ES = false, bool COH = false,
          typename PT = S, bool XU = false>
__device__ __forceinline__ void sweep_body_pf(const SweepArgs<S>& A, const PT* __restrict__ params,
                                              const PT* __restrict__ etab, const S* __restrict__ ghat,
                                              const double* __restrict__ lanetab,
                                              S* __restrict__ xface, S* __restrict__ yface, S* __restrict__ zface,
                                              S* __restrict__ spec, double* __restrict__ partial,
                                              S* __restrict__ plane, const WorkUnit u)
{
    const int lane = threadIdx.x;
    const int o = u.o, tile = u.tile, I = u.I, J = u.J, K = u.K;
    const bool px = (o & 1) != 0, py = (o & 2) != 0, pz = (o & 4) != 0;
    const int slot = tile * 64 + lane;
    const int nx = A.nx, ny = A.ny, nz = A.nz, MT = A.MT;
    constexpr unsigned SB = sizeof(S), PB = sizeof(PT);
    constexpr bool PD = sizeof(PT) > sizeof(S);  // parameters wider than f
    const size_t fstride = (size_t)A.slots * VL;
    const unsigned lofs = (unsigned)slot * VL * SB;
    // a face cell of this brick, as a 32-bit byte offset from the brick's face
    // base: c <= (BZ - 1) * max(nx, ny) + max(BX, BY) - 1 on the x and y faces,
    // c <= (BY - 1) * nx + BX - 1 on the z face; the host keeps c * rowb below 2^32
    const unsigned rowb = (unsigned)(fstride * SB);
    auto fcell = [rowb](auto* base, int c) { return (decltype(base))((const char*)base + (unsigned)c * rowb); };

    const int iend = min(BX, nx - I * BX), jend = min(BY, ny - J * BY);
    const int kend = min(A.bz, nz - K * A.bz);
    const bool wx = I < A.nbx - 1, wy = J < A.nby - 1, wz = K < A.nbz - 1;
    const int ir0 = I * BX, jr0 = J * BY, kr0 = K * A.bz;
    const int si = px ? 1 : -1, sj = py ? nx : -nx, sk = pz ? nx * ny : -nx * ny;
    const int cell0 = (px ? ir0 : nx - 1 - ir0) + nx * ((py ? jr0 : ny - 1 - jr0) + ny * (pz ? kr0 : nz - 1 - kr0));

    const S* xin = xface + ((size_t)(o * 2 + ((I - 1) & 1)) * nz * ny + (size_t)kr0 * ny + jr0) * fstride;
    S* xout = xface + ((size_t)(o * 2 + (I & 1)) * nz * ny + (size_t)kr0 * ny + jr0) * fstride;
    const S* yin = yface + ((size_t)(o * 2 + ((J - 1) & 1)) * nz * nx + (size_t)kr0 * nx + ir0) * fstride;
    S* yout = yface + ((size_t)(o * 2 + (J & 1)) * nz * nx + (size_t)kr0 * nx + ir0) * fstride;
    const S* zin = zface + ((size_t)(o * 2 + ((K - 1) & 1)) * ny * nx + (size_t)jr0 * nx + ir0) * fstride;
    S* zout = zface + ((size_t)(o * 2 + (K & 1)) * ny * nx + (size_t)jr0 * nx + ir0) * fstride;
    S* sbuf = A.spec_on ? spec + (size_t)(o & 3) * ny * nx * fstride : nullptr;
    const S* xgin = nullptr; S* xgout = nullptr;
    const S* ygin = nullptr; S* ygout = nullptr;
    const S* zgin = nullptr; S* zgout = nullptr;
    S* sgbuf = nullptr;
    if constexpr (O2) {
        xgin = A.xgface + (xin - xface);
        xgout = A.xgface + (xout - xface);
        ygin = A.ygface + (yin - yface);
        ygout = A.ygface + (yout - yface);
        zgin = A.zgface + (zin - zface);
        zgout = A.zgface + (zout - zface);
        sgbuf = A.spec_on ? A.specg + (size_t)(o & 3) * ny * nx * fstride : nullptr;
    }

    auto lds = [&](int jj, int ii, int v) -> S& { return plane[((jj * BX + ii) * VL + v) * 64 + lane]; };
    // the z inflow of the last row's last two cells in registers (ZR = 2):
    // their slots are the last two of the f plane, and of the F plane that
    // follows it directly at second order (zr0/zr1 hold f, zg0/zg1 F);
    // the launch does not allocate them
    constexpr int ZR = zreg_cells<S, VL, BX, BY, O2, ES, COH>();
    auto ldz = [&](int jj, int ii, int v) -> S& {
        return plane[((BY * BX - ZR + jj * BX + ii) * VL + v) * 64 + lane];
    };
    S zr0[VL], zr1[VL], zg0[VL], zg1[VL];
#pragma unroll
    for (int v = 0; v < VL; ++v) zr0[v] = zr1[v] = zg0[v] = zg1[v] = (S)0;
    auto zreg = [&](int jj, int ii) { return ZR == 2 && jj == BY - 1 && ii >= BX - 2; };

    // ---- lane constants
    const double* lt = lanetab + ((size_t)o * A.slots + slot) * A.lstride;
    const double xiy_d = lt[0], xiz_d = lt[1];
    const S xiy = (S)xiy_d, xiz = (S)xiz_d;
    const S ay = (S)lt[2], az = (S)lt[3];
    const int vb = (int)lt[4], vc = (int)lt[5];
    // |xi_x| / h_x is formed per cell from the node and a wave-uniform
    // factor (the octant's sign over h_x, or the sign alone on a non-uniform
    // mesh, whose cells bring their own inverse size): fewer live registers
    S xix[VL];
    double xd[VL], wd[VL];
    // first order, FP32 storage: the lane's x-moment weights w, w xi_x,
    // w xi_x^2, w xi_x^3 of each velocity, so that each moment sum takes one
    // FMA per velocity (FP64 storage gains nothing from it, being bound by
    // memory, and its dependency-driven form has no registers left for it)
    constexpr bool WP = !O2 && !PD && sizeof(S) == 4;
    double wx1[VL], wx2[VL], wx3[VL];
    unsigned oa[VL], oal[VL];
#pragma unroll
    for (int v = 0; v < VL; ++v) {
        xd[v] = lt[LT_SHARED + LT_PER_V * v + 0];
        wd[v] = lt[LT_SHARED + LT_PER_V * v + 2];
        const int a = (int)lt[LT_SHARED + LT_PER_V * v + 3];
        xix[v] = (S)xd[v];
        oa[v] = (unsigned)a * PB;
        oal[v] = (unsigned)(a + A.mx * (vb + A.my * vc)) * SB;
        wx1[v] = wd[v] * xd[v];
        wx2[v] = wx1[v] * xd[v];
        wx3[v] = wx2[v] * xd[v];
    }
    const unsigned ob = (unsigned)(A.mx + vb) * PB, oc = (unsigned)(A.mx + A.my + vc) * PB;
    const S sgx = px ? (S)A.rdx : -(S)A.rdx;
    const double yz2 = xiy_d * xiy_d + xiz_d * xiz_d;
    const int sideX = px ? 0 : 1, sideY = py ? 2 : 3, sideZ = pz ? 4 : 5;
    const int shX = 4 * sideX, shY = 4 * sideY, shZ = 4 * sideZ;
    const int ridx = reduce13_index(lane);
    const bool writer = (lane & 3) == 0;  // one lane per slot 0..15 of the record
    // second order on a stretched mesh: the slope weights of this octant's
    // direction along each axis, per cell index
    const double* thxt = nullptr;
    const double* thyt = nullptr;
    const double* thzt = nullptr;
    if constexpr (O2 && NU) {
        thxt = A.theta + (px ? 0 : nx);
        thyt = A.theta + 2 * nx + (py ? 0 : ny);
        thzt = A.theta + 2 * nx + 2 * ny + (pz ? 0 : nz);
    }
    const unsigned oridx = (unsigned)ridx * 8u;
    double* part = partial + ((size_t)(o * A.ntiles + tile) * A.N) * PREC;

    // ---- the first plane's z inflow: the upwind brick's outflow face
    if (kr0 > 0) {
        for (int jj = 0; jj < jend; ++jj)
            for (int ii = 0; ii < iend; ++ii) {
                S t[VL];
                load_face<COH>(zin, (unsigned)(jj * nx + ii) * rowb, lofs, t);
                if (zreg(jj, ii)) {
                    if (ii == BX - 1) {
#pragma unroll
                        for (int v = 0; v < VL; ++v) zr1[v] = t[v];
                    } else {
#pragma unroll
                        for (int v = 0; v < VL; ++v) zr0[v] = t[v];
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < VL; ++v) lds(jj, ii, v) = t[v];
                }
                if constexpr (O2) {
                    load_face<COH>(zgin, (unsigned)(jj * nx + ii) * rowb, lofs, t);
                    if (zreg(jj, ii)) {
                        if (ii == BX - 1) {
#pragma unroll
                            for (int v = 0; v < VL; ++v) zg1[v] = t[v];
                        } else {
#pragma unroll
                            for (int v = 0; v < VL; ++v) zg0[v] = t[v];
                        }
                    } else {
#pragma unroll
                        for (int v = 0; v < VL; ++v) ldz(jj, ii, v) = t[v];
                    }
                }
            }
    }

    // ---- loads of the next cell, issued one cell ahead
    PT eb_n = (PT)0, ec_n = (PT)0, ex_n[VL];
    S fx_n[VL], fy_n[VL];
    // second order: F of the x / y faces; for the second row fy_n holds the
    // f of the row behind the y face (the same face value the first row took)
    S gx_n[VL], gy_n[VL];
#pragma unroll
    for (int v = 0; v < VL; ++v) {
        ex_n[v] = (PT)0;
        fx_n[v] = fy_n[v] = gx_n[v] = gy_n[v] = (S)0;
    }
    // the next cell's record is read one cell ahead as well: its info word
    // and 1/tau (which also bring the record's first cache lines into the
    // scalar cache for the rest of its loads)
    PT nu_n = (PT)1;
    uint32_t info_n = 0;
    auto prefetch = [&](int ii, int jj, int kk) {
        const int cn = cell0 + ii * si + jj * sj + kk * sk;
        const PT* Pn = params + (size_t)cn * PSTRIDE;
        nu_n = Pn[P_NU];
        info_n = reinterpret_cast<const uint32_t*>(Pn + P_INFO)[0];
        const PT* E = etab + (size_t)cn * MT;
        eb_n = ldg(E, ob);
        ec_n = ldg(E, oc);
#pragma unroll
        for (int v = 0; v < VL; ++v) ex_n[v] = ldg(E, oa[v]);
        if (ii == 0 && ir0 > 0) {
            load_face<COH>(xin, (unsigned)(kk * ny + jj) * rowb, lofs, fx_n);
            if constexpr (O2) load_face<COH>(xgin, (unsigned)(kk * ny + jj) * rowb, lofs, gx_n);
        }
        if ((jj == 0 || (O2 && jj == 1)) && jr0 > 0) {
            load_face<COH>(yin, (unsigned)(kk * nx + ii) * rowb, lofs, fy_n);
        }
        if constexpr (O2) {
            if (jj == 0 && jr0 > 0) {
                load_face<COH>(ygin, (unsigned)(kk * nx + ii) * rowb, lofs, gy_n);
            }
        }
    };

    const int ncell = iend * jend * kend;
    int ii = 0, jj = 0, kk = 0;
    prefetch(0, 0, 0);
    S prev[VL], prevF[VL];
#pragma unroll
    for (int v = 0; v < VL; ++v) prev[v] = prevF[v] = (S)0;
    uint32_t ybnd = 0;  // second order: plane cells whose y upwind side is a boundary
    // the last fluid cell whose stores are pending (pcell < 0: none; in the
    // second-order form only its moment record, its faces being out)
    int pcell = -1, pii = 0, pjj = 0, pkk = 0;
    double ptot = 0.0;
    S pFy[VL], pFz[VL];
#pragma unroll
    for (int v = 0; v < VL; ++v) pFy[v] = pFz[v] = (S)0;
    auto flush_faces = [&]() {
        if (pcell < 0) return;
        if (pii == BX - 1 && wx) {
            store_face<COH>(xout, (unsigned)(pkk * ny + pjj) * rowb, lofs, prev);
            if constexpr (O2) {
                store_face<COH>(xgout, (unsigned)(pkk * ny + pjj) * rowb, lofs, prevF);
            }
        }
        if (pjj == BY - 1 && wy) {
            store_face<COH>(yout, (unsigned)(pkk * nx + pii) * rowb, lofs, prev);
            if constexpr (O2) {
                store_face<COH>(ygout, (unsigned)(pkk * nx + pii) * rowb, lofs, pFy);
            }
        }
        if (pkk == A.bz - 1 && wz) {
            store_face<COH>(zout, (unsigned)(pjj * nx + pii) * rowb, lofs, prev);
            if constexpr (O2) {
                store_face<COH>(zgout, (unsigned)(pjj * nx + pii) * rowb, lofs, pFz);
            }
        }
        if (sbuf != nullptr && !pz && kr0 + pkk == nz - 1) {
            const int i = px ? ir0 + pii : nx - 1 - (ir0 + pii);
            const int j = py ? jr0 + pjj : ny - 1 - (jr0 + pjj);
            store_face<false>(sbuf + ((size_t)j * nx + i) * fstride, 0u, lofs, prev);
            if constexpr (O2) {
                store_face<false>(sgbuf + ((size_t)j * nx + i) * fstride, 0u, lofs, pFz);
            }
        }
    };
    auto flush_partial = [&]() {
        if (pcell >= 0 && writer) stb_nt(part + (size_t)pcell * PREC, oridx, ptot);
    };
    auto flush = [&]() {
        flush_faces();
        flush_partial();
    };
    for (int n = 0; n < ncell; ++n) {
        const PT eb = eb_n, ec = ec_n, nu = nu_n;
        const uint32_t info = info_n;
        PT ex[VL];
        S fxp[VL], fyp[VL], gxp[VL], gyp[VL];
#pragma unroll
        for (int v = 0; v < VL; ++v) {
            ex[v] = ex_n[v];
            fxp[v] = fx_n[v];
            fyp[v] = fy_n[v];
            gxp[v] = gx_n[v];
            gyp[v] = gy_n[v];
        }
        if (O2 && ii == 0 && jj == 0) ybnd = 0;
        int ni = ii + 1, nj = jj, nk = kk;
        if (ni == iend) {
            ni = 0;
            if (++nj == jend) {
                nj = 0;
                ++nk;
            }
        }
        // the loads issued one cell ahead are in (vmcnt 0; the other
        // counters left alone): nothing issued before this point is waited
        // for later in the cell
        wait_vector_memory();

        const int cell = cell0 + ii * si + jj * sj + kk * sk;
        const PT* P = params + (size_t)cell * PSTRIDE;
        // second order: the weight of this cell's own slope in the value
        // it carries through its downstream face along each axis, h / (h +
        // h_up) (1/2 on a uniform mesh), and that of the row behind along y
        S thx = (S)0.5, thy = (S)0.5, thz = (S)0.5, thyb = (S)0.5;
        if constexpr (O2 && NU) {
            const int ri = px ? ir0 + ii : nx - 1 - (ir0 + ii);
            const int rj = py ? jr0 + jj : ny - 1 - (jr0 + jj);
            const int rk = pz ? kr0 + kk : nz - 1 - (kr0 + kk);
            thx = (S)thxt[ri];
            thy = (S)thyt[rj];
            thz = (S)thzt[rk];
            if (jj > 0) thyb = (S)thyt[py ? rj - 1 : rj + 1];
        }
        if (!(info & SOLID_BIT)) {
            S fx[VL], fy[VL], fz[VL];
            S ux[VL], uy[VL], uz[VL];
            bool ixf = false, iyf = false, izf = false;
            {
                const uint32_t code = (info >> shX) & 15u;
                if (code == 0) {
                    if constexpr (O2) {
                        ixf = true;
#pragma unroll
                        for (int v = 0; v < VL; ++v) {
                            ux[v] = ii > 0 ? S(prev[v]) : S(fxp[v]);
                            fx[v] = (ii > 0 ? S(prevF[v]) : S(gxp[v])) + thx * ux[v];
                        }
                    } else {
#pragma unroll
                        for (int v = 0; v < VL; ++v) fx[v] = ii > 0 ? prev[v] : fxp[v];
                    }
                } else {
                    const S rf = (S)P[P_RHO_SIDE + sideX];
                    const S* g = ghat + (size_t)(code - 1) * A.NV;
#pragma unroll
                    for (int v = 0; v < VL; ++v) fx[v] = rf * ldg(g, oal[v]);
                }
            }
            {
                const uint32_t code = (info >> shY) & 15u;
                if constexpr (O2) {
                    if (code != 0) ybnd |= 1u << (jj * BX + ii);
                }
                if (code == 0) {
                    if constexpr (O2) {
                        iyf = true;
                        if (jj > 0) {
                            // F of the row behind, rebuilt from its own upwind row
                            const bool edge = (ybnd >> ((jj - 1) * BX + ii)) & 1u;
#pragma unroll
                            for (int v = 0; v < VL; ++v) {
                                const S fu = lds(jj - 1, ii, v);
                                const S f2 = jj >= 2 ? S(lds(jj - 2, ii, v)) : S(fyp[v]);
                                uy[v] = fu;
                                fy[v] = (edge ? fu : ((S)1 + thyb) * fu - thyb * f2) + thy * fu;
                            }
                        } else {
#pragma unroll
                            for (int v = 0; v < VL; ++v) {
                                uy[v] = fyp[v];
                                fy[v] = gyp[v] + thy * fyp[v];
                            }
                        }
                    } else if (jj > 0) {
                        // the row behind as an opaque scalar: its values
                        // are then read at small positive offsets from one
                        // address (derived from this row's address, they
                        // would sit at negative offsets, one address each)
                        int rowy = (jj - 1) * BX + ii;
                        asm("" : "+s"(rowy));
#pragma unroll
                        for (int v = 0; v < VL; ++v) fy[v] = plane[(rowy * VL + v) * 64 + lane];
                    } else {
#pragma unroll
                        for (int v = 0; v < VL; ++v) fy[v] = fyp[v];
                    }
                } else {
                    const S rf = (S)P[P_RHO_SIDE + sideY];
                    const S* g = ghat + (size_t)(code - 1) * A.NV;
#pragma unroll
                    for (int v = 0; v < VL; ++v) fy[v] = rf * ldg(g, oal[v]);
                }
            }
            {
                const uint32_t code = (info >> shZ) & 15u;
                // the interior inflow is read from LDS whatever the cell's
                // side: a boundary alternative then loads after it, never
                // before it on a path the compiler has to assume (a load
                // ahead of the LDS read into the same registers makes it
                // wait for every load in flight, those issued one cell
                // ahead included)
                S zl[VL], zg[VL];
                if (zreg(jj, ii)) {
                    if (ii == BX - 1) {
#pragma unroll
                        for (int v = 0; v < VL; ++v) {
                            zl[v] = zr1[v];
                            zg[v] = O2 ? zg1[v] : (S)0;
                        }
                    } else {
#pragma unroll
                        for (int v = 0; v < VL; ++v) {
                            zl[v] = zr0[v];
                            zg[v] = O2 ? zg0[v] : (S)0;
                        }
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < VL; ++v) {
                        zl[v] = lds(jj, ii, v);
                        zg[v] = O2 ? S(ldz(jj, ii, v)) : (S)0;
                    }
                }
                // pinned here: not moved below the loads of the branches
                // (first order; the second-order form has no registers to spare)
                if constexpr (!O2) {
#pragma unroll
                    for (int v = 0; v < VL; ++v) keep_alive(zl[v]);
                }
                if (O2 && code == 0) {
                    izf = true;
#pragma unroll
                    for (int v = 0; v < VL; ++v) {
                        uz[v] = zl[v];
                        fz[v] = zg[v] + thz * uz[v];
                    }
                } else if (O2 && code == CODE_SPECULAR) {
                    // the mirror image beyond the symmetry plane
                    izf = true;
                    const int i = px ? ir0 + ii : nx - 1 - (ir0 + ii);
                    const int j = py ? jr0 + jj : ny - 1 - (jr0 + jj);
                    const S* src = sbuf + ((size_t)j * nx + i) * fstride;
                    const S* gsrc = sgbuf + ((size_t)j * nx + i) * fstride;
#pragma unroll
                    for (int v = 0; v < VL; ++v) {
                        uz[v] = ldb(src, lofs + v * SB);
                        fz[v] = ldb(gsrc, lofs + v * SB) + (S)0.5 * uz[v];
                    }
                } else if (code == 0) {
#pragma unroll
                    for (int v = 0; v < VL; ++v) fz[v] = zl[v];
                } else if (code == CODE_SPECULAR) {
                    const int i = px ? ir0 + ii : nx - 1 - (ir0 + ii);
                    const int j = py ? jr0 + jj : ny - 1 - (jr0 + jj);
                    const S* src = sbuf + ((size_t)j * nx + i) * fstride;
#pragma unroll
                    for (int v = 0; v < VL; ++v) fz[v] = ldb(src, lofs + v * SB);
                } else {
                    const S rf = (S)P[P_RHO_SIDE + sideZ];
                    const S* g = ghat + (size_t)(code - 1) * A.NV;
#pragma unroll
                    for (int v = 0; v < VL; ++v) fz[v] = rf * ldg(g, oal[v]);
                }
            }

            // first order: the previous cell's stores and the next cell's
            // loads go out once the inflow is resolved (its boundary loads
            // waited for here): no wait below then covers them
            if constexpr (!O2) {
                wait_vector_memory();
                flush();
                if (n + 1 < ncell) prefetch(ni, nj, nk);
            }

            const PT Ux = P[P_UX], Uy = P[P_UY], Uz = P[P_UZ];
            const PT L0 = P[P_L0], L1 = P[P_L1], L2 = P[P_L2], L3 = P[P_L3], L4 = P[P_L4];
            const PT qx = P[P_QX], qy = P[P_QY], qz = P[P_QZ], tT = P[P_TWO_T];
            const PT gyz = eb * ec;
            const PT cy = (PD ? (PT)xiy_d : (PT)xiy) - Uy, cz = (PD ? (PT)xiz_d : (PT)xiz) - Uz;
            const PT cyz2 = cy * cy + cz * cz;
            const PT Lyz = L0 + L2 * cy + L3 * cz;
            const PT Qyz = qy * cy + qz * cz;
            // ES-BGK: qx, qy, qz hold A_xy, A_xz, A_yz
            const PT Bes = qx * cy + qy * cz, Ces = qz * cy * cz;
            PT xn[VL];
#pragma unroll
            for (int v = 0; v < VL; ++v) xn[v] = PD ? (PT)xd[v] : (PT)xix[v];
            EsCross<PT, ES && XU && sizeof(PT) == 8 && (VL > 1)> cross(xn[0], xn[VL > 1 ? 1 : 0], Ux, Bes, Ces);
            // upwind coefficients: lane constants |xi_d| / h_d (uniform mesh),
            // or |xi_d| times the cell's inverse sizes (non-uniform mesh)
            S ayc = ay, azc = az, sx = sgx;
            if constexpr (NU) {
                sx = sgx * (S)P[P_IDX];
                ayc = ay * (S)P[P_IDY];
                azc = az * (S)P[P_IDZ];
            }
            const S aynu = ayc + azc + (S)nu;
            double u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
            double e0 = 0.0, e1 = 0.0, e2 = 0.0;  // second order: sum w (F_d - f)
            S Fy[VL], Fz[VL];
            const S kx = O2 && ixf ? (S)1 + thx : (S)1, ky = O2 && iyf ? (S)1 + thy : (S)1;
            const S kz = O2 && izf ? (S)1 + thz : (S)1;
            const S ayk = ayc * ky, azk = azc * kz;
            // FP64 ES-BGK: one reciprocal for the lane's denominators (in
            // the Shakhov and second-order forms the products' registers
            // would spill or cost a wave per SIMD)
            constexpr bool BR = sizeof(S) == 8 && VL > 1 && ES && !O2;
            double rden[VL];
            if constexpr (BR) {
                double dd[VL];
#pragma unroll
                for (int v = 0; v < VL; ++v) {
                    const S axv = xix[v] * sx;
                    dd[v] = O2 ? double(axv * kx + ayk + azk + (S)nu) : double(axv + aynu);
                }
                batch_rcp<VL>(dd, rden);
            }
#pragma unroll
            for (int v = 0; v < VL; ++v) {
                const PT cx = (PD ? (PT)xd[v] : (PT)xix[v]) - Ux;
                const PT c2 = cx * cx + cyz2;
                PT nfs;
                if constexpr (ES) {
                    nfs = gyz * ex[v] * (Lyz + L1 * cx + L4 * c2) * cross.at(v, xn[v], xn[v > 0 ? v - 1 : 0], cx, Bes, Ces);
                } else {
                    const PT poly = Lyz + L1 * cx + L4 * c2 + (Qyz + qx * cx) * (c2 * tT - (PT)5);
                    nfs = gyz * ex[v] * poly;
                }
                const S axv = xix[v] * sx;
                const S num = axv * fx[v] + ayc * fy[v] + azc * fz[v] + (S)nfs;
                S f;
                if constexpr (O2) {
                    if constexpr (BR)
                        f = num * (S)rden[v];
                    else
                        f = num * fast_rcp(axv * kx + ayk + azk + (S)nu);
                    const S dx = ixf ? thx * (f - ux[v]) : (S)0;
                    const S dy = iyf ? thy * (f - uy[v]) : (S)0;
                    const S dz = izf ? thz * (f - uz[v]) : (S)0;
                    prevF[v] = f + dx;
                    Fy[v] = f + dy;
                    Fz[v] = f + dz;
                    if (!zreg(jj, ii))
                        ldz(jj, ii, v) = Fz[v];
                    else if (ii == BX - 1)
                        zg1[v] = Fz[v];
                    else
                        zg0[v] = Fz[v];
                    e0 += wd[v] * xd[v] * (double)dx;
                    e1 += wd[v] * (double)dy;
                    e2 += wd[v] * (double)dz;
                } else {
                    if constexpr (BR)
                        f = num * (S)rden[v];
                    else
                        f = num * fast_rcp(axv + aynu);
                }
                prev[v] = f;
                if (!zreg(jj, ii))
                    lds(jj, ii, v) = f;
                else if (ii == BX - 1)
                    zr1[v] = f;
                else
                    zr0[v] = f;
                if constexpr (WP) {
                    const double fd = (double)f;
                    u0 = fma(wd[v], fd, u0);
                    u1 = fma(wx1[v], fd, u1);
                    u2 = fma(wx2[v], fd, u2);
                    u3 = fma(wx3[v], fd, u3);
                } else {
                    const double t0 = wd[v] * (double)f;
                    const double t1 = t0 * xd[v];
                    const double t2 = t1 * xd[v];
                    u0 += t0;
                    u1 += t1;
                    u2 += t2;
                    u3 += t2 * xd[v];
                }
            }
            if constexpr (O2) {
                // second order: the previous cell's moment record and this
                // cell's faces go out now, the next cell's loads after them
                // (the wait at the top of the next cell then finds all of
                // them issued a reduction earlier)
                flush_partial();
                pcell = cell;
                pii = ii;
                pjj = jj;
                pkk = kk;
#pragma unroll
                for (int v = 0; v < VL; ++v) {
                    pFy[v] = Fy[v];
                    pFz[v] = Fz[v];
                }
                flush_faces();
                if (n + 1 < ncell) prefetch(ni, nj, nk);
            }

            double m[O2 ? 16 : 13];
            m[0] = u0;
            m[1] = u1;
            m[2] = xiy_d * u0;
            m[3] = xiz_d * u0;
            m[4] = u2;
            m[5] = xiy_d * m[2];
            m[6] = xiz_d * m[3];
            m[7] = xiy_d * u1;
            m[8] = xiz_d * u1;
            m[9] = xiz_d * m[2];
            m[10] = u3 + yz2 * u1;
            const double t2 = u2 + yz2 * u0;
            m[11] = xiy_d * t2;
            m[12] = xiz_d * t2;
            double tot;
            if constexpr (O2) {
                m[13] = e0;
                m[14] = xiy_d * e1;
                m[15] = xiz_d * e2;
                tot = wave_reduce16(m);
            } else {
                tot = wave_reduce13(m);
            }
            // first order: the cell's stores go out in the next cell, after
            // the wait for the loads issued one cell ahead and before the
            // next ones: a store between a load and its wait would be waited
            // for as well (one in-order counter covers loads and stores)
            pcell = cell;
            pii = ii;
            pjj = jj;
            pkk = kk;
            ptot = tot;
        } else {
            if constexpr (O2)
                flush_partial();  // its faces are out
            else
                flush();
            if (n + 1 < ncell) prefetch(ni, nj, nk);
            pcell = -1;
        }
        ii = ni;
        jj = nj;
        kk = nk;
    }
    if constexpr (O2)
        flush_partial();  // its faces are out
    else
        flush();
}

// NU: non-uniform mesh (the upwind coefficients take the cell's own sizes).
// Occupancy with 4 per lane: 4 waves per SIMD (128 registers) in FP32, 3
// (168) in FP64, reached without spills inside the cell loop.
// PT: see sweep_body_pf (the parameter record and tables are of type PT).
template <typename S, int VL, int BX, int BY, bool NU, typename PT = S>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(VL == 4 ? (sizeof(S) == 4 && sizeof(PT) == 4 ? 4 : 3) : 1)))
void sweep_kernel_pf(const SweepArgs<S> A)
{
    S* plane = reinterpret_cast<S*>(dvm_sweep_lds);
    sweep_body_pf<S, VL, BX, BY, NU, false, false, false, PT>(
        A, reinterpret_cast<const PT*>(A.params), reinterpret_cast<const PT*>(A.etab), A.ghat, A.lanetab, A.xface,
        A.yface, A.zface, A.spec, A.partial, plane, diagonal_unit(A, A.bricks));
}

// Spin until the three upwind bricks of a work unit (those that exist) have
// published this launch's epoch.  The wait is bounded: it gives up after
// DYN_WAIT_TICKS of the 100 MHz real-time counter (half a second), or at
// once when another wave has already given up (the launch is then reported
// as failed and its iterate discarded, so no wave needs to wait any more).
constexpr unsigned long long DYN_WAIT_TICKS = 50000000ull;
__device__ __forceinline__ bool wait_upwind(const unsigned* fx, const unsigned* fy, const unsigned* fz,
                                            unsigned epoch, const int* errflag)
{
    unsigned long long t0 = 0;
    for (unsigned n = 0;; ++n) {
        const unsigned a = fx ? __hip_atomic_load(fx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : epoch;
        const unsigned b = fy ? __hip_atomic_load(fy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : epoch;
        const unsigned c = fz ? __hip_atomic_load(fz, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : epoch;
        if (a == epoch && b == epoch && c == epoch) return true;
        const unsigned long long now = __builtin_amdgcn_s_memrealtime();
        if (n == 0) t0 = now;
        if (now - t0 > DYN_WAIT_TICKS) return false;
        if (__hip_atomic_load(errflag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 8) return false;
        __builtin_amdgcn_s_sleep(2);
    }
}

// Dependency-driven form of the same sweep: one launch covers every brick
// diagonal of the octants in A (all of one velocity group, or one specular
// phase).  Each wave takes work units from a device-wide counter in the
// order (diagonal, brick, octant, tile) -- every unit's upwind bricks come
// earlier in that order and were taken by waves that are already running,
// so every wait ends -- waits until its three upwind bricks of the same
// octant and tile have published this launch's epoch, sweeps the brick,
// waits for its own stores and publishes.  Faces move through
// device-coherent loads and stores (load_face / store_face with COH), the ready
// flags through relaxed device-scope atomics; the counter is never reset:
// the host passes the value it held before the launch (every wave ends with
// one failed take, so a launch of G waves advances it by units + G).
template <typename S, int VL, int BX, int BY, bool NU, typename PT = S>
__global__ __launch_bounds__(64)
__attribute__((amdgpu_waves_per_eu(VL == 4 ? (sizeof(S) == 4 && sizeof(PT) == 4 ? 4 : 3) : 1)))
void sweep_kernel_dyn(const SweepArgs<S> Aarg)
{
    S* plane = reinterpret_cast<S*>(dvm_sweep_lds);
    for (;;) {
        // the arguments are read afresh from the kernel-argument segment in
        // every work unit (through an opaque copy of its address): hoisted
        // out of the loop they would stay live in registers across the whole
        // brick and spill
        using KArgs = const __attribute__((address_space(4))) SweepArgs<S>;
        KArgs* Ap = (KArgs*)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(Ap));
        const SweepArgs<S>& A = *(const SweepArgs<S>*)Ap;
        const int per_brick = A.noct * A.ntiles;
        const int nbx = A.nbx, nby = A.nby, nbz = A.nbz;
        const size_t chain = (size_t)nbx * nby * nbz;  // flags of one (octant, tile)
        unsigned long long t = 0;
        if (threadIdx.x == 0) t = __hip_atomic_fetch_add(A.head, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)t);
        const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(t >> 32));
        const long long item = (long long)((((unsigned long long)hi << 32) | lo) - A.qbase);
        if (item >= (long long)A.nitems) break;
        const int b = (int)(item / per_brick), r = (int)(item % per_brick);
        WorkUnit u;
        u.o = A.oct_base + r / A.ntiles;
        u.tile = r % A.ntiles;
        u.I = A.bricks[4 * b + 0];
        u.J = A.bricks[4 * b + 1];
        u.K = A.bricks[4 * b + 2];
        unsigned* f = A.ready + ((size_t)u.o * A.ntiles + u.tile) * chain;
        const size_t self = ((size_t)u.K * nby + u.J) * nbx + u.I;
        if (!wait_upwind(u.I > 0 ? f + self - 1 : nullptr, u.J > 0 ? f + self - nbx : nullptr,
                         u.K > 0 ? f + self - (size_t)nbx * nby : nullptr, A.epoch, A.errflag)) {
            if (threadIdx.x == 0) atomicOr(A.errflag, 8);
        }
        asm volatile("" ::: "memory");
        sweep_body_pf<S, VL, BX, BY, NU, false, false, true, PT>(
            A, reinterpret_cast<const PT*>(A.params), reinterpret_cast<const PT*>(A.etab), A.ghat, A.lanetab, A.xface,
            A.yface, A.zface, A.spec, A.partial, plane, u);
        // the brick's face stores are complete before its flag says so
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __hip_atomic_store(f + self, A.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename S, int VL, int BX, int BY, bool NU>
__global__ __launch_bounds__(64) void sweep_kernel(const SweepArgs<S> A)
{
    S* plane = reinterpret_cast<S*>(dvm_sweep_lds);
    sweep_body<S, VL, BX, BY, NU>(A, A.params, A.etab, A.ghat, A.lanetab, A.bricks, A.xface, A.yface, A.zface,
                              A.spec, A.partial, plane);
}

// second-order upwind and/or ES-BGK (uniform meshes), pipelined body
// (occupancy: FP32 ES-BGK with 4 per lane fits 4 waves per SIMD without
// spills in the loop; the FP64 and second-order forms would spill there)
template <typename S, int VL, int BX, int BY, bool O2, bool ES, bool NU = false, bool XU = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(VL == 4 && !O2 && sizeof(S) == 4 ? 4 : 1)))
void sweep_kernel_pfx(const SweepArgs<S> A)
{
    S* plane = reinterpret_cast<S*>(dvm_sweep_lds);
    sweep_body_pf<S, VL, BX, BY, NU, O2, ES, false, S, XU>(A, A.params, A.etab, A.ghat, A.lanetab, A.xface,
                                                           A.yface, A.zface, A.spec, A.partial, plane,
                                                           diagonal_unit(A, A.bricks));
}

// second-order upwind and/or ES-BGK (uniform meshes, plain body)
template <typename S, int VL, int BX, int BY, bool O2, bool ES>
__global__ __launch_bounds__(64) void sweep_kernel_x(const SweepArgs<S> A)
{
    S* plane = reinterpret_cast<S*>(dvm_sweep_lds);
    sweep_body<S, VL, BX, BY, false, O2, ES>(A, A.params, A.etab, A.ghat, A.lanetab, A.bricks, A.xface,
                                             A.yface, A.zface, A.spec, A.partial, plane);
}

// instantiated variants: (precision, VL, BX, BY)
#define DVM_SWEEP_VARIANTS(X) \
    X(double, 1, 4, 4) X(double, 2, 4, 4) X(double, 2, 4, 2) X(double, 4, 4, 2) X(double, 4, 4, 4) \
    X(double, 2, 2, 2) X(double, 4, 2, 2) X(double, 4, 3, 2) \
    X(float, 1, 4, 4) X(float, 2, 4, 4) X(float, 2, 4, 2) X(float, 4, 4, 2) X(float, 4, 4, 4) \
    X(float, 4, 2, 2) X(float, 8, 4, 2) X(float, 8, 2, 2)
// the shapes the defaults choose, also built for non-uniform meshes
#define DVM_SWEEP_VARIANTS_NU(X) \
    X(double, 1, 4, 4) X(double, 2, 4, 2) X(double, 4, 4, 2) X(double, 4, 3, 2) \
    X(float, 1, 4, 4) X(float, 2, 4, 2) X(float, 4, 4, 2)
// and for the second-order and ES-BGK sweeps
// (3x2 bricks: the pipelined first-order ES-BGK sweep in FP64, the
// pipelined second-order Shakhov sweep in FP32)
#define DVM_SWEEP_VARIANTS_O2(X) \
    X(double, 1, 4, 4) X(double, 2, 4, 2) X(double, 4, 2, 2) X(double, 4, 4, 2) X(double, 4, 3, 2) \
    X(float, 1, 4, 4) X(float, 2, 4, 2) X(float, 4, 4, 2) X(float, 4, 3, 2)

bool sweep_variant_available(int prec, int vl, int bx, int by, int nonuniform, int order2, int esbgk)
{
#define X(T, V, BXX, BYY) \
    if ((prec == 0) == (sizeof(T) == 8) && vl == V && bx == BXX && by == BYY) return true;
    if (order2 || esbgk) {
        // on a stretched mesh: pipelined body with two or more velocities
        // per lane; 3x2 bricks for the first-order ES-BGK sweep in FP64 and
        // the second-order Shakhov sweep in FP32 only
        if (nonuniform && vl < 2) return false;
        if (bx == 3 && (prec == 0 ? (order2 || !esbgk) : (!order2 || esbgk))) return false;
        DVM_SWEEP_VARIANTS_O2(X)
    } else if (nonuniform) {
        DVM_SWEEP_VARIANTS_NU(X)
    } else {
        DVM_SWEEP_VARIANTS(X)
    }
#undef X
    return false;
}

template <typename T, int V, int BXX, int BYY, bool NU, typename PT = T>
hipError_t launch_sweep_t(int pipelined, const void* args, hipStream_t st)
{
    const SweepArgs<T>& a = *(const SweepArgs<T>*)args;
    const int zr = pipelined == 1 ? zreg_cells<T, V, BXX, BYY, false, false, false>() : 0;
    const size_t lds = (size_t)(BYY * BXX - zr) * V * 64 * sizeof(T);
    if (pipelined == 2) {
        // as many waves as stay resident (more would only wait for a CU)
        static thread_local int resident = 0, cached_dev = -1;
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        if (resident == 0 || cached_dev != dev) {
            int per_cu = 0, cus = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sweep_kernel_dyn<T, V, BXX, BYY, NU, PT>, 64,
                                                             lds);
            if (e != hipSuccess) return e;
            e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return e;
            resident = std::max(1, per_cu) * std::max(1, cus);
            cached_dev = dev;
        }
        const int grid = std::min(resident, a.nitems);
        sweep_kernel_dyn<T, V, BXX, BYY, NU, PT><<<grid, 64, lds, st>>>(a);
        e = hipGetLastError();
        if (e == hipSuccess) *a.launched = grid;
        return e;
    }
    if (pipelined)
        sweep_kernel_pf<T, V, BXX, BYY, NU, PT><<<a.nblocks, 64, lds, st>>>(a);
    else if constexpr (sizeof(PT) == sizeof(T))
        sweep_kernel<T, V, BXX, BYY, NU><<<a.nblocks, 64, lds, st>>>(a);
    else
        return hipErrorInvalidValue;  // the plain body has no wider parameters
    return hipGetLastError();
}

template <typename T, int V, int BXX, int BYY>
hipError_t launch_sweep_x(int pipelined, int order2, int esbgk, int nonuniform, const void* args, hipStream_t st)
{
    const SweepArgs<T>& a = *(const SweepArgs<T>*)args;
    // the plane of f, and with the second order the plane of F along z (the
    // pipelined second-order Shakhov body keeps zreg_cells of each in registers)
    const int zr = pipelined && order2 && !esbgk ? zreg_cells<T, V, BXX, BYY, true, false, false>() : 0;
    const size_t lds = ((size_t)(order2 ? 2 : 1) * BYY * BXX - 2 * zr) * V * 64 * sizeof(T);
    // FP64 ES-BGK on a uniform x axis: the cross factors by recurrence
    constexpr bool XR = sizeof(T) == 8 && V > 1;
    const bool xr = XR && esbgk && a.xuni;
    // 3x2 bricks: built for the pipelined sweeps whose LDS plane would hold
    // them below the waves their registers allow -- in FP64 the first-order
    // ES-BGK form, in FP32 the second-order Shakhov form
    constexpr bool ES_ONLY = BXX == 3 && sizeof(T) == 8, O2_ONLY = BXX == 3 && sizeof(T) == 4;
    if (ES_ONLY && (order2 || !esbgk || !pipelined)) return hipErrorInvalidValue;
    if (O2_ONLY && (!order2 || esbgk || !pipelined)) return hipErrorInvalidValue;
    if (nonuniform) {
        // stretched mesh: pipelined body, two or more velocities per lane
        if (!pipelined || V < 2) return hipErrorInvalidValue;
        if constexpr (V < 2) {
            return hipErrorInvalidValue;
        } else if constexpr (O2_ONLY) {
            sweep_kernel_pfx<T, V, BXX, BYY, true, false, true><<<a.nblocks, 64, lds, st>>>(a);
        } else if constexpr (ES_ONLY) {
            if (xr)
                sweep_kernel_pfx<T, V, BXX, BYY, false, true, true, XR><<<a.nblocks, 64, lds, st>>>(a);
            else
                sweep_kernel_pfx<T, V, BXX, BYY, false, true, true><<<a.nblocks, 64, lds, st>>>(a);
        } else {
            if (order2 && esbgk && xr)
                sweep_kernel_pfx<T, V, BXX, BYY, true, true, true, XR><<<a.nblocks, 64, lds, st>>>(a);
            else if (order2 && esbgk)
                sweep_kernel_pfx<T, V, BXX, BYY, true, true, true><<<a.nblocks, 64, lds, st>>>(a);
            else if (order2)
                sweep_kernel_pfx<T, V, BXX, BYY, true, false, true><<<a.nblocks, 64, lds, st>>>(a);
            else if (xr)
                sweep_kernel_pfx<T, V, BXX, BYY, false, true, true, XR><<<a.nblocks, 64, lds, st>>>(a);
            else
                sweep_kernel_pfx<T, V, BXX, BYY, false, true, true><<<a.nblocks, 64, lds, st>>>(a);
        }
        return hipGetLastError();
    }
    if (pipelined) {
        if constexpr (O2_ONLY) {
            sweep_kernel_pfx<T, V, BXX, BYY, true, false><<<a.nblocks, 64, lds, st>>>(a);
        } else if constexpr (ES_ONLY) {
            if (xr)
                sweep_kernel_pfx<T, V, BXX, BYY, false, true, false, XR><<<a.nblocks, 64, lds, st>>>(a);
            else
                sweep_kernel_pfx<T, V, BXX, BYY, false, true><<<a.nblocks, 64, lds, st>>>(a);
        } else {
            if (order2 && esbgk && xr)
                sweep_kernel_pfx<T, V, BXX, BYY, true, true, false, XR><<<a.nblocks, 64, lds, st>>>(a);
            else if (order2 && esbgk)
                sweep_kernel_pfx<T, V, BXX, BYY, true, true><<<a.nblocks, 64, lds, st>>>(a);
            else if (order2)
                sweep_kernel_pfx<T, V, BXX, BYY, true, false><<<a.nblocks, 64, lds, st>>>(a);
            else if (xr)
                sweep_kernel_pfx<T, V, BXX, BYY, false, true, false, XR><<<a.nblocks, 64, lds, st>>>(a);
            else
                sweep_kernel_pfx<T, V, BXX, BYY, false, true><<<a.nblocks, 64, lds, st>>>(a);
        }
        return hipGetLastError();
    }
    if constexpr (ES_ONLY || O2_ONLY) {
        return hipErrorInvalidValue;
    } else {
        if (order2 && esbgk)
            sweep_kernel_x<T, V, BXX, BYY, true, true><<<a.nblocks, 64, lds, st>>>(a);
        else if (order2)
            sweep_kernel_x<T, V, BXX, BYY, true, false><<<a.nblocks, 64, lds, st>>>(a);
        else
            sweep_kernel_x<T, V, BXX, BYY, false, true><<<a.nblocks, 64, lds, st>>>(a);
        return hipGetLastError();
    }
}

bool sweep_wide_params_available(int prec, int vl, int bx, int by, int nonuniform, int order2, int esbgk)
{
    return prec == 1 && vl == 4 && bx == 4 && by == 2 && !nonuniform && !order2 && !esbgk;
}

hipError_t launch_sweep(int prec, int vl, int bx, int by, int pipelined, int nonuniform, int order2,
                        int esbgk, int wide_params, const void* args, hipStream_t st)
{
    if (wide_params) {
        if (!sweep_wide_params_available(prec, vl, bx, by, nonuniform, order2, esbgk) || pipelined == 0)
            return hipErrorInvalidValue;
        return launch_sweep_t<float, 4, 4, 2, false, double>(pipelined, args, st);
    }
    if (order2 || esbgk) {
#define X(T, V, BXX, BYY)                                                     \
        if ((prec == 0) == (sizeof(T) == 8) && vl == V && bx == BXX && by == BYY) \
            return launch_sweep_x<T, V, BXX, BYY>(pipelined, order2, esbgk, nonuniform, args, st);
        DVM_SWEEP_VARIANTS_O2(X)
#undef X
        return hipErrorInvalidValue;
    }
#define X(T, V, BXX, BYY)                                                                  \
    if ((prec == 0) == (sizeof(T) == 8) && vl == V && bx == BXX && by == BYY)              \
        return launch_sweep_t<T, V, BXX, BYY, NUV>(pipelined, args, st);
    if (nonuniform) {
#define NUV true
        DVM_SWEEP_VARIANTS_NU(X)
#undef NUV
    } else {
#define NUV false
        DVM_SWEEP_VARIANTS(X)
#undef NUV
    }
#undef X
    return hipErrorInvalidValue;
}

// --------------------------------------------------------------------------
// A5: finalisation
// --------------------------------------------------------------------------

__global__ __launch_bounds__(256) void finalize_kernel(Consts C, DevPtrs D, const double* __restrict__ partial,
                                                       int ntiles, const double* __restrict__ gout,
                                                       double* __restrict__ Wn, double* __restrict__ qn,
                                                       double* __restrict__ rwn, double* __restrict__ stress_n,
                                                       double* __restrict__ blockmass, int* __restrict__ flag)
{
    __shared__ double red[256];
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = C.N;
    double mass = 0.0;
    if (cell < N) {
        const uint32_t info = D.cellinfo[cell];
        if (info & SOLID_BIT) {
            for (int v = 0; v < 5; ++v) Wn[(size_t)v * N + cell] = 0.0;
            for (int v = 0; v < 3; ++v) qn[(size_t)v * N + cell] = 0.0;
            for (int s = 0; s < 6; ++s) rwn[(size_t)s * N + cell] = 0.0;
            if (C.esbgk)
                for (int s = 0; s < 6; ++s) stress_n[(size_t)s * N + cell] = 0.0;
        } else {
            double m[13];
            for (int k = 0; k < 13; ++k) m[k] = 0.0;
            double hp[3] = {0, 0, 0}, hm[3] = {0, 0, 0};  // half-range mass fluxes
            for (int o = 0; o < 8; ++o) {
                double g1 = 0, g2 = 0, g3 = 0;
                for (int t = 0; t < ntiles; ++t) {
                    const double* p = partial + ((size_t)(o * ntiles + t) * N + cell) * PREC;
#pragma unroll
                    for (int k = 0; k < 13; ++k) m[k] += p[k];
                    g1 += p[1];
                    g2 += p[2];
                    g3 += p[3];
                    if (C.order2) {
                        // second order: what crosses the downstream faces
                        g1 += p[13];
                        g2 += p[14];
                        g3 += p[15];
                    }
                }
                if (o & 1) hp[0] += g1; else hm[0] += g1;
                if (o & 2) hp[1] += g2; else hm[1] += g2;
                if (o & 4) hp[2] += g3; else hm[2] += g3;
            }
            const double rho = m[0];
            if (!(rho > 0.0) || !isfinite(rho)) atomicOr(flag, 4);
            const double Ux = m[1] / rho, Uy = m[2] / rho, Uz = m[3] / rho;
            const double trM = m[4] + m[5] + m[6];
            Wn[cell] = rho;
            Wn[(size_t)N + cell] = m[1];
            Wn[(size_t)2 * N + cell] = m[2];
            Wn[(size_t)3 * N + cell] = m[3];
            Wn[(size_t)4 * N + cell] = 0.5 * trM;
            // q_i = 1/2 sum w c_i |c|^2 f, c = xi - U^{n+1}, expanded in raw moments
            const double U[3] = {Ux, Uy, Uz};
            const double U2 = Ux * Ux + Uy * Uy + Uz * Uz;
            const double Mij[3][3] = {{m[4], m[7], m[8]}, {m[7], m[5], m[9]}, {m[8], m[9], m[6]}};
            for (int d = 0; d < 3; ++d) {
                const double UM = Mij[d][0] * Ux + Mij[d][1] * Uy + Mij[d][2] * Uz;
                const double val = m[10 + d] - 2.0 * UM - U[d] * trM + 2.0 * rho * U[d] * U2;
                qn[(size_t)d * N + cell] = 0.5 * val;
            }
            if (C.esbgk) {
                // stress per unit mass about U^{n+1}: M_ij / rho - U_i U_j
                stress_n[cell] = m[4] / rho - Ux * Ux;
                stress_n[(size_t)N + cell] = m[5] / rho - Uy * Uy;
                stress_n[(size_t)2 * N + cell] = m[6] / rho - Uz * Uz;
                stress_n[(size_t)3 * N + cell] = m[7] / rho - Ux * Uy;
                stress_n[(size_t)4 * N + cell] = m[8] / rho - Ux * Uz;
                stress_n[(size_t)5 * N + cell] = m[9] / rho - Uy * Uz;
            }
            for (int s = 0; s < 6; ++s) {
                const uint32_t code = (info >> (4 * s)) & 15u;
                double r = 0.0;
                if (code != 0 && code != CODE_SPECULAR && C.kind_wall[code - 1]) {
                    const int d = s >> 1;
                    // particles hitting side s move along -n: s odd (upper) -> xi_d > 0
                    const double flux = (s & 1) ? hp[d] : -hm[d];
                    r = flux / gout[(code - 1) * 6 + s];
                }
                rwn[(size_t)s * N + cell] = r;
            }
            const int i = cell % C.nx, j = (cell / C.nx) % C.ny, k = cell / (C.nx * C.ny);
            mass = rho * (D.h[i] * D.h[C.nx + j] * D.h[C.nx + C.ny + k]);
        }
    }
    red[threadIdx.x] = mass;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) blockmass[blockIdx.x] = red[0];
}

hipError_t launch_finalize(const Consts& C, const DevPtrs& D, const double* partial, int ntiles,
                           const double* gout, double* Wn, double* qn, double* rwn, double* stress_n,
                           double* blockmass, int nblocks, int* flag, hipStream_t st)
{
    finalize_kernel<<<nblocks, 256, 0, st>>>(C, D, partial, ntiles, gout, Wn, qn, rwn, stress_n, blockmass, flag);
    return hipGetLastError();
}

// Velocity groups: the records of one group's tiles summed per octant and
// cell, in tile order, into the accumulator that finalize reads as a single
// tile.  One thread per (octant, cell, record slot): a 16-thread group reads
// one 128-byte record line.
__global__ __launch_bounds__(256) void fold_kernel(const double* __restrict__ partial, int ntiles, int N,
                                                   int add, double* __restrict__ acc)
{
    const size_t n = (size_t)8 * N * PREC;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t rec = i / PREC;  // o * N + cell
    const int k = (int)(i % PREC);
    const size_t o = rec / N, cell = rec % N;
    double s = add ? acc[i] : 0.0;
    for (int t = 0; t < ntiles; ++t) s += partial[((o * ntiles + t) * N + cell) * PREC + k];
    acc[i] = s;
}

hipError_t launch_fold(const double* partial, int ntiles, int N, int add, double* acc, hipStream_t st)
{
    const size_t n = (size_t)8 * N * PREC;
    const unsigned nb = (unsigned)((n + 255) / 256);
    fold_kernel<<<nb, 256, 0, st>>>(partial, ntiles, N, add, acc);
    return hipGetLastError();
}

// deterministic block sum of n values (fixed strided order + fixed tree)
__device__ double block_sum_fixed(const double* x, int n, double* red)
{
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += x[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void scale_residual_kernel(Consts C, DevPtrs D, double M0,
                                                             const double* __restrict__ blockmass, int nbm,
                                                             double* __restrict__ Wn, double* __restrict__ qn,
                                                             double* __restrict__ rwn, const double* __restrict__ Wo,
                                                             double* __restrict__ respart)
{
    __shared__ double red[256];
    const double total = block_sum_fixed(blockmass, nbm, red);
    const double s = C.closed ? M0 / total : 1.0;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = C.N;
    double dd[5] = {0, 0, 0, 0, 0}, nn[5] = {0, 0, 0, 0, 0};
    if (cell < N && !(D.cellinfo[cell] & SOLID_BIT)) {
        for (int v = 0; v < 5; ++v) {
            const double w = Wn[(size_t)v * N + cell] * s;
            Wn[(size_t)v * N + cell] = w;
            const double d = w - Wo[(size_t)v * N + cell];
            dd[v] = d * d;
            nn[v] = w * w;
        }
        if (C.closed) {
            for (int v = 0; v < 3; ++v) qn[(size_t)v * N + cell] *= s;
            for (int v = 0; v < 6; ++v) rwn[(size_t)v * N + cell] *= s;
        }
    }
    for (int v = 0; v < 10; ++v) {
        red[threadIdx.x] = v < 5 ? dd[v] : nn[v - 5];
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) respart[(size_t)blockIdx.x * 10 + v] = red[0];
        __syncthreads();
    }
}

hipError_t launch_scale_residual(const Consts& C, const DevPtrs& D, double M0, const double* blockmass,
                                 int nbm, double* Wn, double* qn, double* rwn, const double* Wo,
                                 double* respart, int nblocks, hipStream_t st)
{
    scale_residual_kernel<<<nblocks, 256, 0, st>>>(C, D, M0, blockmass, nbm, Wn, qn, rwn, Wo, respart);
    return hipGetLastError();
}

// out[0..4]: residual per field, out[5]: total mass before rescaling,
// out[6]: error flag
__global__ __launch_bounds__(256) void residual_final_kernel(const double* __restrict__ respart, int nblocks,
                                                             const double* __restrict__ blockmass, int nbm,
                                                             double* __restrict__ out, const int* __restrict__ flag)
{
    __shared__ double red[256];
    double vals[10];
    for (int v = 0; v < 10; ++v) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s += respart[(size_t)b * 10 + v];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        vals[v] = red[0];
        __syncthreads();
    }
    const double mass = block_sum_fixed(blockmass, nbm, red);
    if (threadIdx.x == 0) {
        for (int v = 0; v < 5; ++v) {
            const double dn = vals[v], nn = vals[5 + v];
            out[v] = nn > 0 ? sqrt(dn / nn) : (dn > 0 ? sqrt(dn) : 0.0);
        }
        out[5] = mass;
        out[6] = (double)(*flag);
    }
}

hipError_t launch_residual_final(const double* respart, int nblocks, const double* blockmass, int nbm,
                                 double* out, const int* flag, hipStream_t st)
{
    residual_final_kernel<<<1, 256, 0, st>>>(respart, nblocks, blockmass, nbm, out, flag);
    return hipGetLastError();
}

}  // namespace dvm
