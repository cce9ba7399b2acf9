// Host runtime of libdvm_hip.so: the C ABI declared in include/dvm.h.
//
// The runtime owns no device memory: the caller lends one workspace and the
// runtime carves it into the buffers below.  Each outer iteration is a fixed
// sequence of launches on the context's stream (parameters, one sweep launch
// per brick diagonal, finalisation, rescaling/residual) followed by one
// 64-byte device-to-host copy of the residual, which is the only host
// synchronisation per iteration.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "dvm.h"
#include "dvm_internal.h"

using namespace dvm;

namespace {

thread_local std::string g_err;

dvm_status fail(dvm_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(DVM_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct dvm_ctx {
    dvm_grid g;
    dvm_vgrid vg;
    dvm_gas gas;
    int prec;
    hipStream_t stream;
    dvm_face_bc faces[6];
    std::vector<uint8_t> solid;
    double solid_u[3] = {0, 0, 0};
    double solid_T = 1.0;
    int closed = 1;

    // derived
    int N = 0, NV = 0, nfluid = 0;
    double dx[3];
    int hsplit[3];  // number of nodes with xi < 0 along each axis
    int VL = 2, BX = 4, BY = 4, BZ = 8;
    int PF = 1;  // sweep body: 0 plain, 1 software-pipelined, 2 pipelined and dependency-driven
    // schedule requested with dvm_set_schedule (0: the library's choice);
    // req_ok is false while the request names a kernel shape that is not
    // built for the current precision, mesh kind, order and model
    int req_vl = 0, req_bx = 0, req_by = 0, req_bz = 0, req_body = 0;
    bool req_ok = true;
    bool fits32 = true;  // the 32-bit face offsets of the schedule fit
    int order = 1;  // spatial order of the upwind scheme (1 or 2)
    // FP32 storage with the parameter record, Gaussian tables and the
    // equilibrium evaluation in FP64 (dvm_set_parameter_precision(ctx, 64))
    bool wide = false;
    int pprec() const { return wide ? DVM_F64 : prec; }  // type of params and tables
    int model = 0;  // 0: Shakhov, 1: ES-BGK
    // velocity nodes and weights per axis (empty: uniform, trapezoid)
    std::vector<double> vnode[3], vweight[3];
    std::vector<double> h[3];  // cell sizes along x, y, z (empty: uniform)
    std::vector<double> hstage;  // host copy of the uploaded sizes
    std::vector<double> thstage; // host copy of the uploaded second-order slope weights
    bool nonuniform = false;
    int nbx = 0, nby = 0, nbz = 0;
    int ntiles = 0, slots = 0, lstride = 0;
    // velocity groups: each octant's tiles split into ngroups consecutive
    // ranges, swept one after another (faces, mirror planes and partials
    // sized for one range; the moments folded into acc between ranges)
    int groups_req = 1, ngroups = 1, gtiles = 0;
    std::vector<int> gt0;  // first tile of each group, plus ntiles at the end
    std::vector<int> bricks;           // I, J, K, 0 per brick, grouped by diagonal
    std::vector<int> diag_off, diag_cnt;
    int ndiag = 0;
    bool spec_on = false;

    // workspace
    char* ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    int static_dev = -1;  // device whose static workspace is bound (-1: a lent one)
    struct {
        size_t axes, spacing, cellinfo, bricks, lanetab, kstate, ghat, ghat64, gout, W, q, rw, params, etab,
            partial, acc, xface, yface, zface, spec, xg, yg, zg, specg, stress, blockmass, respart, out, flag,
            ready, head, theta, end;
    } off;
    size_t Ssz = 8;
    int nbF = 0;  // blocks of the per-cell kernels (256 threads)

    // dependency-driven sweep: epoch of the last launch (ready flags hold
    // it) and the work-unit counter's value before the next launch
    unsigned epoch = 0;
    unsigned long long qbase = 0;

    // state
    int cur = 0;
    bool initialized = false;
    double M0 = 0;
    double res[5] = {0, 0, 0, 0, 0};
    std::vector<uint32_t> cellinfo;
    double kind_rho[8] = {0};
    int kind_wall[8] = {0};

    // the per-diagonal sweep launches of disjoint octant sets go to separate
    // streams (forked from and joined back into `stream` around the sweep):
    // the octants are independent within an iteration, so one set's next
    // diagonal fills the device while another's launch drains
    int nstreams = 2;
    hipStream_t sub[8] = {};
    hipEvent_t fork_ev = nullptr, join_ev[8] = {};

    // timing (level 2 also times every sweep launch on its own stream)
    int timing = 0;
    std::vector<hipEvent_t> lev;  // launch events: start, end per launch
    double t_launch = 0;
    long long n_launch = 0;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    double t_params = 0, t_sweep = 0, t_final = 0;
    int t_iters = 0;

    template <typename T>
    T* P(size_t o) const { return reinterpret_cast<T*>(ws + o); }
};

// The allocation-free workspace: one array per device, lent to at most one
// context at a time by dvm_bind_static_workspace.  In host code `scratch` is
// only a handle for the runtime's symbol lookup; its device address on each
// device comes from hipGetSymbolAddress with that device current.
constexpr size_t kStaticWorkspaceBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};
const dvm_ctx* g_static_owner[kMaxDevices] = {};

// a context bound to a device's static workspace may touch it only while it
// is that workspace's latest owner
dvm_status check_workspace_owner(const dvm_ctx* c)
{
    if (c->static_dev < 0) return DVM_OK;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_owner[c->static_dev] != c)
        return fail(DVM_ERR_STATE, "the static workspace of device %d was bound to another context since",
                    c->static_dev);
    return DVM_OK;
}

void derive_schedule(dvm_ctx* c)
{
    c->N = c->g.nx * c->g.ny * c->g.nz;
    c->NV = c->vg.m[0] * c->vg.m[1] * c->vg.m[2];
    c->dx[0] = c->g.lx / c->g.nx;
    c->dx[1] = c->g.ly / c->g.ny;
    c->dx[2] = c->g.lz / c->g.nz;
    for (int d = 0; d < 3; ++d) c->hsplit[d] = c->vg.m[d] / 2;
    c->Ssz = c->prec == DVM_F64 ? 8 : 4;

    // velocities per lane, brick shape and body: the library's choice, or
    // what dvm_set_schedule requested where that kernel is built.
    // VL: 4 velocities per lane, halved while more than 1/8 of the lanes'
    // velocity slots of the larger x half would be empty.  Brick and body by
    // measurement (cavity 64^3 x 32^3 FP64, 96^3 x 28^3 and cube FP32):
    // 4x2 bricks and the software-pipelined body (FP64 with 4 per lane,
    // whose first-order Shakhov body keeps two cells of the 4x2 plane in
    // registers so that 3 waves per SIMD stay resident: 64^3 x 32^3 307
    // GPt/s against 289 at 3x2, which moves a third more x-face traffic; on
    // the mesh stretched 1.02 per cell 302 against 289, the paper cube 318
    // against 303; the FP64 ES-BGK body keeps its whole plane in LDS and
    // takes 3x2 bricks, whose 12 KB plane lets in the 3 waves per SIMD its
    // registers allow: 240 GPt/s against 230 at 4x2; likewise the
    // second-order FP32 form, whose two 8 KB planes 3x2 brings to 12 KB:
    // 96^3 x 28^3 251 against 232); the second-order FP64
    // form takes 2 per lane
    // and 4x2 bricks (141 GPt/s against 131 with 4 per lane at 2x2, the most
    // its registers and two LDS planes allow); 1 per lane: plain body, 4x4.
    const int nax = c->vg.m[0] - c->hsplit[0];  // larger half along x
    const bool f64 = c->prec == DVM_F64;
    const int o2 = c->order == 2, es = c->model == 1;
    int vl = 4;
    // FP64 takes 4 per lane in the first-order forms (96^3 x 28^3, 14 nodes
    // per half: 263 GPt/s against 257 with 2 per lane, whose 22 tiles per
    // octant write 70 % more moment records than 13), 2 at second order
    if (f64 && o2) vl = 2;
    while (vl > 1 && 8 * (((nax + vl - 1) / vl) * vl - nax) > ((nax + vl - 1) / vl) * vl) vl /= 2;
    auto default_bx = [&](int v) {
        return v != 4 ? 4 : f64 ? (o2 ? 2 : es ? 3 : 4) : (o2 && !es ? 3 : 4);
    };
    auto default_by = [&](int v) { return v == 1 ? 4 : 2; };
    if (!sweep_variant_available(c->prec, vl, default_bx(vl), default_by(vl), c->nonuniform, o2, es)) vl = 1;
    int bx = default_bx(vl), by = default_by(vl);
    int pf = vl >= 2 ? 1 : 0;
    // cells per brick column: 16 for the FP64 sweeps with 2 or 4 per lane
    // (cavity 64^3 x 32^3 with the launches on two streams, 4x2 bricks:
    // 303-307 GPt/s against 305-307 at 12, 299 at 20, 296 at 24, 278 at 32;
    // on the 1.02-stretched mesh 300 against 296 at 12; second order 151
    // against 145 at 12, ES-BGK 205 against 203; 96^3 x 28^3 with 2 per
    // lane 255 against 250 at 8), 12 for the FP32 ones with 4 per lane (cube
    // 510 against 499 at 8 and 502 at 10; 96^3 x 28^3 426 against 422 at 8
    // and 425 at 16, second order 231 against 227), 8 otherwise
    int bz = f64 ? (vl >= 2 ? 16 : 8) : (vl == 4 ? 12 : 8);
    c->req_ok = true;
    if (c->req_vl || c->req_bx || c->req_by || c->req_bz || c->req_body) {
        const int rv = c->req_vl ? c->req_vl : vl;
        const int rbx = c->req_bx ? c->req_bx : (c->req_vl ? default_bx(rv) : bx);
        const int rby = c->req_by ? c->req_by : (c->req_vl ? default_by(rv) : by);
        // the dependency-driven launch exists for the first-order Shakhov sweep
        const bool body_ok = c->req_body != 3 || (!o2 && !es);
        if (body_ok && sweep_variant_available(c->prec, rv, rbx, rby, c->nonuniform, o2, es)) {
            vl = rv;
            bx = rbx;
            by = rby;
            if (c->req_bz) bz = c->req_bz;
            if (c->req_body) pf = c->req_body - 1;
        } else {
            c->req_ok = false;
        }
    }
    c->VL = vl;
    c->BX = bx;
    c->BY = by;
    c->BZ = bz;
    c->PF = pf;
    c->nbx = (c->g.nx + c->BX - 1) / c->BX;
    c->nby = (c->g.ny + c->BY - 1) / c->BY;
    c->nbz = (c->g.nz + c->BZ - 1) / c->BZ;

    // tiles: lanes per octant = ceil(na_x / VL) * na_y * na_z
    int nt = 0;
    for (int o = 0; o < 8; ++o) {
        int na[3];
        for (int d = 0; d < 3; ++d) na[d] = ((o >> d) & 1) ? c->vg.m[d] - c->hsplit[d] : c->hsplit[d];
        const int ng = (na[0] + c->VL - 1) / c->VL;
        const int lanes = ng * na[1] * na[2];
        const int t = (lanes + 63) / 64;
        if (t > nt) nt = t;
    }
    c->ntiles = nt;
    c->slots = nt * 64;
    c->ngroups = std::max(1, std::min(c->groups_req, nt));
    c->gt0.assign(c->ngroups + 1, 0);
    c->gtiles = 0;
    for (int g = 0; g <= c->ngroups; ++g) c->gt0[g] = (int)((long long)nt * g / c->ngroups);
    for (int g = 0; g < c->ngroups; ++g) c->gtiles = std::max(c->gtiles, c->gt0[g + 1] - c->gt0[g]);
    c->lstride = LT_SHARED + LT_PER_V * c->VL;
    if (c->lstride & 1) c->lstride++;
    // the sweep addresses a face cell of its brick by a 32-bit byte offset
    // from the brick's face base: the x and y faces up to face cell
    // (BZ - 1) * max(nx, ny) + max(BX, BY) - 1, the z face up to
    // (BY - 1) * nx + BX - 1.  Keep both offsets, in bytes of one group's
    // velocities, below 2^32 (shorter brick columns if needed; a grid that
    // breaches this even with BZ = 1 has face buffers far beyond any device
    // memory)
    {
        const size_t rowb = (size_t)c->gtiles * 64 * c->VL * (c->prec == DVM_F64 ? 8 : 4);
        const size_t span = (size_t)std::max(c->g.nx, c->g.ny);
        const size_t zcells = (size_t)(c->BY - 1) * c->g.nx + c->BX;
        auto fits = [&](int bz) {
            const size_t xycells = (size_t)(bz - 1) * span + (size_t)std::max(c->BX, c->BY);
            return std::max(xycells, zcells) * rowb < ((size_t)1 << 32);
        };
        while (c->BZ > 1 && !fits(c->BZ)) c->BZ = std::max(1, c->BZ / 2);
        c->nbz = (c->g.nz + c->BZ - 1) / c->BZ;
        c->fits32 = fits(c->BZ);
    }

    // bricks grouped by diagonal I + J + K
    c->ndiag = c->nbx + c->nby + c->nbz - 2;
    c->bricks.clear();
    c->diag_off.assign(c->ndiag, 0);
    c->diag_cnt.assign(c->ndiag, 0);
    for (int T = 0; T < c->ndiag; ++T) {
        c->diag_off[T] = (int)(c->bricks.size() / 4);
        for (int K = 0; K < c->nbz; ++K)
            for (int J = 0; J < c->nby; ++J) {
                const int I = T - J - K;
                if (I < 0 || I >= c->nbx) continue;
                c->bricks.push_back(I);
                c->bricks.push_back(J);
                c->bricks.push_back(K);
                c->bricks.push_back(0);
            }
        c->diag_cnt[T] = (int)(c->bricks.size() / 4) - c->diag_off[T];
    }
    c->nbF = (c->N + 255) / 256;
}

// cell size along axis d of index i
double cell_size(const dvm_ctx* c, int d, int i) { return c->nonuniform ? c->h[d][i] : c->dx[d]; }

double cell_volume(const dvm_ctx* c, size_t cell)
{
    const int nx = c->g.nx, ny = c->g.ny;
    const int i = (int)(cell % nx), j = (int)((cell / nx) % ny), k = (int)(cell / ((size_t)nx * ny));
    return cell_size(c, 0, i) * cell_size(c, 1, j) * cell_size(c, 2, k);
}

void layout(dvm_ctx* c)
{
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t N = (size_t)c->N, S = c->Ssz;
    // faces, mirror planes and partials hold one velocity group
    const size_t fst = (size_t)c->gtiles * 64 * c->VL;
    c->off.axes = take(sizeof(double) * (2 * 3 + 5) * MAXM);
    c->off.spacing = take(sizeof(double) * (size_t)(c->g.nx + c->g.ny + c->g.nz));
    c->off.cellinfo = take(sizeof(uint32_t) * N);
    c->off.bricks = take(sizeof(int) * c->bricks.size());
    c->off.lanetab = take(sizeof(double) * 8 * (size_t)c->slots * c->lstride);
    c->off.kstate = take(sizeof(double) * 4 * NKIND);
    c->off.ghat = take(S * NKIND * (size_t)c->NV);
    c->off.ghat64 = take(sizeof(double) * NKIND * (size_t)c->NV);
    c->off.gout = take(sizeof(double) * 6 * NKIND);
    c->off.W = take(sizeof(double) * 2 * 5 * N);
    c->off.q = take(sizeof(double) * 2 * 3 * N);
    c->off.rw = take(sizeof(double) * 2 * 6 * N);
    const size_t SP = c->wide ? sizeof(double) : S;  // parameter record and tables
    c->off.params = take(SP * PSTRIDE * N);
    c->off.etab = take(SP * (size_t)(c->vg.m[0] + c->vg.m[1] + c->vg.m[2]) * N);
    c->off.partial = take(sizeof(double) * PREC * 8 * (size_t)c->gtiles * N);
    c->off.acc = take(c->ngroups > 1 ? sizeof(double) * PREC * 8 * N : 0);
    c->off.xface = take(S * 8 * 2 * (size_t)c->g.nz * c->g.ny * fst);
    c->off.yface = take(S * 8 * 2 * (size_t)c->g.nz * c->g.nx * fst);
    c->off.zface = take(S * 8 * 2 * (size_t)c->g.ny * c->g.nx * fst);
    c->off.spec = take(c->spec_on ? S * 4 * (size_t)c->g.ny * c->g.nx * fst : 0);
    // second order: the F layer of every face buffer and of the mirror plane
    const bool o2 = c->order == 2;
    c->off.xg = take(o2 ? c->off.yface - c->off.xface : 0);
    c->off.yg = take(o2 ? c->off.zface - c->off.yface : 0);
    c->off.zg = take(o2 ? c->off.spec - c->off.zface : 0);
    c->off.specg = take(o2 && c->spec_on ? S * 4 * (size_t)c->g.ny * c->g.nx * fst : 0);
    // ES-BGK: the stress per unit mass, double-buffered like W
    c->off.stress = take(c->model == 1 ? sizeof(double) * 2 * 6 * N : 0);
    c->off.blockmass = take(sizeof(double) * c->nbF);
    c->off.respart = take(sizeof(double) * 10 * c->nbF);
    c->off.out = take(sizeof(double) * 8);
    c->off.flag = take(sizeof(int) * 4);
    c->off.ready = take(c->PF == 2 ? sizeof(unsigned) * 8 * (size_t)c->gtiles * c->nbx * c->nby * c->nbz : 0);
    c->off.head = take(c->PF == 2 ? sizeof(unsigned long long) : 0);
    // second order on a stretched mesh: the slope weights per axis, direction and index
    c->off.theta = take(c->order == 2 && c->nonuniform ? sizeof(double) * 2 * (size_t)(c->g.nx + c->g.ny + c->g.nz)
                                                         : 0);
    c->off.end = o;
}

Consts make_consts(const dvm_ctx* c)
{
    Consts C;
    memset(&C, 0, sizeof C);
    C.nx = c->g.nx;
    C.ny = c->g.ny;
    C.nz = c->g.nz;
    C.N = c->N;
    C.mx = c->vg.m[0];
    C.my = c->vg.m[1];
    C.mz = c->vg.m[2];
    C.MT = C.mx + C.my + C.mz;
    C.NV = c->NV;
    const double w = c->gas.omega;
    const double kappa = 15.0 * sqrt(M_PI) / ((5.0 - 2.0 * w) * (7.0 - 2.0 * w));
    C.kappa_kn = kappa * c->gas.kn;
    C.omega = w;
    C.pr = c->gas.pr;
    C.correct = c->gas.conservative_correction;
    C.closed = c->closed;
    C.order2 = c->order == 2;
    C.esbgk = c->model == 1;
    C.xuniform = c->vnode[0].empty() ? 1 : 0;
    for (int k = 0; k < 8; ++k) {
        C.kind_rho[k] = c->kind_rho[k];
        C.kind_wall[k] = c->kind_wall[k];
    }
    return C;
}

DevPtrs make_ptrs(const dvm_ctx* c)
{
    DevPtrs D;
    D.xi = c->P<double>(c->off.axes);
    D.wt = c->P<double>(c->off.axes) + 3 * MAXM;
    D.xmom = c->P<double>(c->off.axes) + 6 * MAXM;
    D.cellinfo = c->P<uint32_t>(c->off.cellinfo);
    D.bricks = c->P<int>(c->off.bricks);
    D.lanetab = c->P<double>(c->off.lanetab);
    D.h = c->P<double>(c->off.spacing);
    return D;
}

void build_cellinfo(dvm_ctx* c)
{
    const int nx = c->g.nx, ny = c->g.ny, nz = c->g.nz;
    c->cellinfo.assign(c->N, 0);
    for (int s = 0; s < 6; ++s) {
        c->kind_wall[s] = c->faces[s].kind == DVM_BC_WALL;
        c->kind_rho[s] = c->faces[s].kind == DVM_BC_FREE ? c->faces[s].rho : 0.0;
    }
    c->kind_wall[6] = 1;
    c->kind_rho[6] = 0.0;
    c->nfluid = 0;
    auto is_solid = [&](int i, int j, int k) {
        return !c->solid.empty() && c->solid[i + nx * (j + ny * k)] != 0;
    };
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int id = i + nx * (j + ny * k);
                uint32_t info = 0;
                if (is_solid(i, j, k)) {
                    info = SOLID_BIT;
                } else {
                    c->nfluid++;
                    for (int s = 0; s < 6; ++s) {
                        int p[3] = {i, j, k};
                        const int ext[3] = {nx, ny, nz};
                        const int d = s >> 1;
                        p[d] += (s & 1) ? 1 : -1;
                        uint32_t code;
                        if (p[d] < 0 || p[d] >= ext[d]) {
                            code = c->faces[s].kind == DVM_BC_SPECULAR ? CODE_SPECULAR : (uint32_t)(s + 1);
                        } else if (is_solid(p[0], p[1], p[2])) {
                            code = 7;
                        } else {
                            code = 0;
                        }
                        info |= code << (4 * s);
                    }
                }
                c->cellinfo[id] = info;
            }
}

std::vector<double> build_lanetab(const dvm_ctx* c, const std::vector<double> xi[3])
{
    // grouped layout: group g holds [8][its slots][lstride], the groups in
    // order (one group: [8][slots][lstride])
    std::vector<double> lt((size_t)8 * c->slots * c->lstride, 0.0);
    for (int o = 0; o < 8; ++o) {
        int na[3];
        bool pos[3];
        for (int d = 0; d < 3; ++d) {
            pos[d] = ((o >> d) & 1) != 0;
            na[d] = pos[d] ? c->vg.m[d] - c->hsplit[d] : c->hsplit[d];
        }
        const int ng = (na[0] + c->VL - 1) / c->VL;
        const int lanes = ng * na[1] * na[2];
        auto node = [&](int d, int local) {
            return pos[d] ? c->hsplit[d] + local : c->hsplit[d] - 1 - local;
        };
        auto weight = [&](int d, int a) {
            if (!c->vweight[d].empty()) return c->vweight[d][a];
            const int M = c->vg.m[d];
            const double h = 2.0 * c->vg.vmax[d] / (M - 1);
            return (a == 0 || a == M - 1) ? 0.5 * h : h;
        };
        for (int s = 0; s < c->slots; ++s) {
            int grp = 0;
            while (s >= 64 * c->gt0[grp + 1]) ++grp;
            const int s0 = 64 * c->gt0[grp], gs = 64 * c->gt0[grp + 1] - s0;
            double* L = &lt[((size_t)8 * s0 + (size_t)o * gs + (s - s0)) * c->lstride];
            const bool lane_on = s < lanes && na[1] > 0 && na[2] > 0 && na[0] > 0;
            const int ss = lane_on ? s : 0;
            int g = 0, bl = 0, cl = 0;
            if (na[0] > 0 && na[1] > 0 && na[2] > 0) {
                g = ss % ng;
                bl = (ss / ng) % na[1];
                cl = ss / (ng * na[1]);
            }
            const int b = na[1] > 0 ? node(1, bl) : 0, cc = na[2] > 0 ? node(2, cl) : 0;
            L[0] = xi[1][b];
            L[1] = xi[2][cc];
            // |xi_d| / h_d; on a non-uniform mesh |xi_d| (the sweep takes the
            // cell's own inverse sizes)
            L[2] = fabs(xi[1][b]) / (c->nonuniform ? 1.0 : c->dx[1]);
            L[3] = fabs(xi[2][cc]) / (c->nonuniform ? 1.0 : c->dx[2]);
            L[4] = b;
            L[5] = cc;
            for (int v = 0; v < c->VL; ++v) {
                int al = g * c->VL + v;
                bool on = lane_on && al < na[0];
                if (al >= na[0]) al = na[0] > 0 ? na[0] - 1 : 0;
                const int a = na[0] > 0 ? node(0, al) : 0;
                double* Lv = L + LT_SHARED + LT_PER_V * v;
                Lv[0] = xi[0][a];
                Lv[1] = fabs(xi[0][a]) / (c->nonuniform ? 1.0 : c->dx[0]);
                Lv[2] = on ? weight(0, a) * weight(1, b) * weight(2, cc) : 0.0;
                Lv[3] = a;
            }
        }
    }
    return lt;
}

dvm_status check_ctx(dvm_ctx* c)
{
    if (!c) return fail(DVM_ERR_ARG, "null context");
    return DVM_OK;
}

// one outer iteration; writes the candidate state into slot 1-cur and the
// residual summary into out[0..7] on the host
dvm_status run_iteration(dvm_ctx* c, double* hout)
{
    const Consts C = make_consts(c);
    const DevPtrs D = make_ptrs(c);
    const int cur = c->cur, nxt = 1 - cur;
    const size_t N = c->N;
    double* W = c->P<double>(c->off.W);
    double* q = c->P<double>(c->off.q);
    double* rw = c->P<double>(c->off.rw);
    int* flag = c->P<int>(c->off.flag);
    hipStream_t st = c->stream;

    HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), st));
    if (c->timing) HIPCHK(hipEventRecord(c->ev[0], st));
    double* stress = c->model == 1 ? c->P<double>(c->off.stress) : nullptr;
    if (c->model == 1)
        HIPCHK(launch_params_es(C, D, W + cur * 5 * N, stress + cur * 6 * N, rw + cur * 6 * N,
                                c->ws + c->off.params, c->ws + c->off.etab, c->prec, flag, st));
    else
        HIPCHK(launch_params(C, D, W + cur * 5 * N, q + cur * 3 * N, rw + cur * 6 * N, c->ws + c->off.params,
                             c->ws + c->off.etab, c->pprec(), flag, st));
    if (c->timing) HIPCHK(hipEventRecord(c->ev[1], st));

    // sweep: one launch per brick diagonal; with a specular plane the
    // octants moving towards it go first so that the others can read their
    // mirror images.  Velocity groups are swept one after another, each
    // group's moments folded into the accumulator before the next reuses the
    // faces and partials.
    const int phases = c->spec_on ? 2 : 1;
    const bool dyn = c->PF == 2;
    const int nbricks = (int)(c->bricks.size() / 4);
    // octants swept per phase, and the streams that share them
    const int oct_phase = c->spec_on ? 4 : 8;
    const int ns = dyn ? 1 : std::min(c->nstreams, oct_phase);
    int nlaunch = 0;
    if (ns > 1 && !c->fork_ev) {
        HIPCHK(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
        for (int k = 0; k < ns; ++k) {
            HIPCHK(hipStreamCreateWithFlags(&c->sub[k], hipStreamNonBlocking));
            HIPCHK(hipEventCreateWithFlags(&c->join_ev[k], hipEventDisableTiming));
        }
    }
    for (int grp = 0; grp < c->ngroups; ++grp) {
    const int t0 = c->gt0[grp], gnt = c->gt0[grp + 1] - t0;
    if (ns > 1) {
        HIPCHK(hipEventRecord(c->fork_ev, st));
        for (int k = 0; k < ns; ++k) HIPCHK(hipStreamWaitEvent(c->sub[k], c->fork_ev, 0));
    }
    for (int sk = 0; sk < ns; ++sk) {
    hipStream_t ss = ns > 1 ? c->sub[sk] : st;
    // with a specular plane each stream keeps a mirror pair (o, o + 4) of
    // octants: the +z one reads the plane its -z partner wrote in phase 0
    for (int ph = 0; ph < phases; ++ph) {
        // per-diagonal launches, or one dependency-driven launch over all
        // bricks (diagonal 0 standing for all of them)
        for (int T = 0; T < (dyn ? 1 : c->ndiag); ++T) {
            const int cnt = dyn ? nbricks : c->diag_cnt[T];
            if (cnt == 0) continue;
            int launched = 0;
            auto fill = [&](auto& a) {
                using S = typename std::remove_pointer<decltype(a.xface)>::type;
                a.params = c->P<S>(c->off.params);
                a.etab = c->P<S>(c->off.etab);
                a.cellinfo = c->P<uint32_t>(c->off.cellinfo);
                a.ghat = c->P<S>(c->off.ghat);
                a.lanetab = c->P<double>(c->off.lanetab) + (size_t)8 * 64 * t0 * c->lstride;
                a.bricks = c->P<int>(c->off.bricks);
                a.xface = c->P<S>(c->off.xface);
                a.yface = c->P<S>(c->off.yface);
                a.zface = c->P<S>(c->off.zface);
                a.spec = c->spec_on ? c->P<S>(c->off.spec) : nullptr;
                const bool o2 = c->order == 2;
                a.xgface = o2 ? c->P<S>(c->off.xg) : nullptr;
                a.ygface = o2 ? c->P<S>(c->off.yg) : nullptr;
                a.zgface = o2 ? c->P<S>(c->off.zg) : nullptr;
                a.specg = o2 && c->spec_on ? c->P<S>(c->off.specg) : nullptr;
                a.partial = c->P<double>(c->off.partial);
                a.theta = c->order == 2 && c->nonuniform ? c->P<double>(c->off.theta) : nullptr;
                a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz; a.N = c->N;
                a.mx = c->vg.m[0]; a.my = c->vg.m[1]; a.MT = C.MT; a.NV = c->NV;
                a.rdx = c->nonuniform ? 1.0 : 1.0 / c->dx[0];
                a.nbx = c->nbx; a.nby = c->nby; a.nbz = c->nbz; a.bz = c->BZ;
                a.ntiles = gnt; a.slots = gnt * 64; a.lstride = c->lstride;
                a.brick_off = dyn ? 0 : c->diag_off[T]; a.brick_cnt = cnt;
                a.oct_base = (c->spec_on ? 4 * ph : 0) + sk * (oct_phase / ns);
                a.noct = oct_phase / ns;
                a.spec_on = c->spec_on ? 1 : 0;
                a.has_solid = c->nfluid < c->N ? 1 : 0;
                a.xuni = c->vnode[0].empty() ? 1 : 0;
                a.nblocks = a.noct * cnt * gnt;
                a.ready = dyn ? c->P<unsigned>(c->off.ready) : nullptr;
                a.head = dyn ? c->P<unsigned long long>(c->off.head) : nullptr;
                a.qbase = c->qbase;
                a.epoch = dyn ? c->epoch + 1 : 0;
                a.nitems = a.nblocks;
                a.errflag = flag;
                a.launched = &launched;
            };
            hipError_t e;
            const size_t li = (size_t)nlaunch * 2;
            if (c->timing == 2) {
                while (c->lev.size() < li + 2) {
                    hipEvent_t ev;
                    HIPCHK(hipEventCreate(&ev));
                    c->lev.push_back(ev);
                }
                HIPCHK(hipEventRecord(c->lev[li], ss));
            }
            if (c->prec == DVM_F64) {
                SweepArgs<double> a;
                fill(a);
                e = launch_sweep(0, c->VL, c->BX, c->BY, c->PF, c->nonuniform, c->order == 2, c->model == 1, 0, &a,
                                 ss);
            } else {
                SweepArgs<float> a;
                fill(a);
                e = launch_sweep(1, c->VL, c->BX, c->BY, c->PF, c->nonuniform, c->order == 2, c->model == 1, c->wide,
                                 &a, ss);
            }
            if (e != hipSuccess) return fail(DVM_ERR_DEVICE, "sweep launch: %s", hipGetErrorString(e));
            if (c->timing == 2) HIPCHK(hipEventRecord(c->lev[li + 1], ss));
            ++nlaunch;
            if (dyn) {
                // every started wave ends with one failed take of the counter
                c->epoch += 1;
                c->qbase += (unsigned long long)cnt * (c->spec_on ? 4 : 8) * gnt + (unsigned long long)launched;
            }
        }
    }
    }
    if (ns > 1) {
        for (int k = 0; k < ns; ++k) {
            HIPCHK(hipEventRecord(c->join_ev[k], c->sub[k]));
            HIPCHK(hipStreamWaitEvent(st, c->join_ev[k], 0));
        }
    }
    if (c->ngroups > 1)
        HIPCHK(launch_fold(c->P<double>(c->off.partial), gnt, c->N, grp > 0, c->P<double>(c->off.acc), st));
    }
    if (c->timing) HIPCHK(hipEventRecord(c->ev[2], st));

    double* blockmass = c->P<double>(c->off.blockmass);
    double* respart = c->P<double>(c->off.respart);
    double* out = c->P<double>(c->off.out);
    const bool folded = c->ngroups > 1;
    HIPCHK(launch_finalize(C, D, c->P<double>(folded ? c->off.acc : c->off.partial), folded ? 1 : c->ntiles,
                           c->P<double>(c->off.gout),
                           W + nxt * 5 * N, q + nxt * 3 * N, rw + nxt * 6 * N,
                           stress ? stress + nxt * 6 * N : nullptr, blockmass, c->nbF, flag, st));
    HIPCHK(launch_scale_residual(C, D, c->M0, blockmass, c->nbF, W + nxt * 5 * N, q + nxt * 3 * N,
                                 rw + nxt * 6 * N, W + cur * 5 * N, respart, c->nbF, st));
    HIPCHK(launch_residual_final(respart, c->nbF, blockmass, c->nbF, out, flag, st));
    if (c->timing) HIPCHK(hipEventRecord(c->ev[3], st));
    HIPCHK(hipMemcpyAsync(hout, out, sizeof(double) * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (c->timing) {
        float a = 0, b = 0, d = 0;
        HIPCHK(hipEventElapsedTime(&a, c->ev[0], c->ev[1]));
        HIPCHK(hipEventElapsedTime(&b, c->ev[1], c->ev[2]));
        HIPCHK(hipEventElapsedTime(&d, c->ev[2], c->ev[3]));
        c->t_params += a;
        c->t_sweep += b;
        c->t_final += d;
        c->t_iters++;
        if (c->timing == 2) {
            for (int k = 0; k < nlaunch; ++k) {
                float t = 0;
                HIPCHK(hipEventElapsedTime(&t, c->lev[2 * k], c->lev[2 * k + 1]));
                c->t_launch += t;
            }
            c->n_launch += nlaunch;
        }
    }
    return DVM_OK;
}

// ES-BGK: the equilibrium stress per unit mass, (T/2) I, of the conserved
// moments W (5 x N, host) into the current stress slot
dvm_status upload_equilibrium_stress(dvm_ctx* c, const double* Wh)
{
    if (c->model != 1) return DVM_OK;
    const size_t N = c->N;
    std::vector<double> P(6 * N, 0.0);
    for (size_t i = 0; i < N; ++i) {
        const double r = Wh[i];
        if ((c->cellinfo[i] & SOLID_BIT) || !(r > 0)) continue;
        const double ux = Wh[N + i] / r, uy = Wh[2 * N + i] / r, uz = Wh[3 * N + i] / r;
        const double T = (Wh[4 * N + i] - 0.5 * r * (ux * ux + uy * uy + uz * uz)) / (0.75 * r);
        for (int k = 0; k < 3; ++k) P[k * N + i] = 0.5 * T;
    }
    HIPCHK(hipMemcpyAsync(c->P<double>(c->off.stress) + (size_t)c->cur * 6 * N, P.data(), sizeof(double) * 6 * N,
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DVM_OK;
}

dvm_status upload_initial(dvm_ctx* c, const std::vector<double>& Wh)
{
    const size_t N = c->N;
    hipStream_t st = c->stream;
    c->cur = 0;
    double* W = c->P<double>(c->off.W);
    double* q = c->P<double>(c->off.q);
    double* rw = c->P<double>(c->off.rw);
    int* flag = c->P<int>(c->off.flag);
    HIPCHK(hipMemcpyAsync(W, Wh.data(), sizeof(double) * 5 * N, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(q, 0, sizeof(double) * 3 * N, st));
    HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), st));
    const Consts C = make_consts(c);
    const DevPtrs D = make_ptrs(c);
    HIPCHK(hipMemsetAsync(rw, 0, sizeof(double) * 6 * N, st));
    HIPCHK(launch_params(C, D, W, q, rw, c->ws + c->off.params, c->ws + c->off.etab, c->pprec(), flag, st));
    HIPCHK(launch_wall_init(C, D, c->ws + c->off.params, c->ws + c->off.etab, c->P<double>(c->off.ghat64),
                            c->P<double>(c->off.gout), rw, c->pprec(), st));
    int hflag = 0;
    HIPCHK(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (hflag) return fail(DVM_ERR_NONPHYSICAL, "non-physical initial state (flag %d)", hflag);
    if (upload_equilibrium_stress(c, Wh.data())) return DVM_ERR_DEVICE;
    double m = 0;
    for (size_t i = 0; i < N; ++i)
        if (!(c->cellinfo[i] & SOLID_BIT)) m += Wh[i] * cell_volume(c, i);
    c->M0 = m;
    for (int v = 0; v < 5; ++v) c->res[v] = 0;
    c->initialized = true;
    return DVM_OK;
}

}  // namespace

extern "C" {

const char* dvm_last_error(void) { return g_err.c_str(); }

dvm_status dvm_create(const dvm_grid* grid, const dvm_vgrid* vgrid, const dvm_gas* gas, int precision,
                      void* hip_stream, dvm_ctx** out)
{
    if (!out) return fail(DVM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!grid || !vgrid || !gas) return fail(DVM_ERR_ARG, "NULL argument");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) return fail(DVM_ERR_ARG, "grid sizes must be >= 1");
    if (!(grid->lx > 0) || !(grid->ly > 0) || !(grid->lz > 0)) return fail(DVM_ERR_ARG, "lengths must be > 0");
    if ((double)grid->nx * grid->ny * grid->nz > 2.0e9) return fail(DVM_ERR_ARG, "too many cells");
    for (int d = 0; d < 3; ++d) {
        if (vgrid->m[d] < 2 || vgrid->m[d] > MAXM) return fail(DVM_ERR_ARG, "velocity nodes must be in [2, %d]", MAXM);
        if (!(vgrid->vmax[d] > 0)) return fail(DVM_ERR_ARG, "vmax must be > 0");
    }
    if (!(gas->kn > 0) || !(gas->pr > 0) || !(gas->omega >= 0) || !(gas->omega < 2.5))
        return fail(DVM_ERR_ARG, "bad gas constants (kn > 0, pr > 0, 0 <= omega < 2.5)");
    if (precision != DVM_F64 && precision != DVM_F32) return fail(DVM_ERR_ARG, "precision must be DVM_F64 or DVM_F32");
    dvm_ctx* c = new dvm_ctx();
    c->g = *grid;
    c->vg = *vgrid;
    c->gas = *gas;
    c->prec = precision;
    c->stream = (hipStream_t)hip_stream;
    for (int s = 0; s < 6; ++s) {
        c->faces[s].kind = DVM_BC_WALL;
        c->faces[s].u[0] = c->faces[s].u[1] = c->faces[s].u[2] = 0.0;
        c->faces[s].T = 1.0;
        c->faces[s].rho = 1.0;
    }
    derive_schedule(c);
    *out = c;
    return DVM_OK;
}

dvm_status dvm_set_face_bc(dvm_ctx* c, int face, const dvm_face_bc* bc)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (c->bound) return fail(DVM_ERR_STATE, "boundary conditions must be set before binding the workspace");
    if (face < 0 || face > 5 || !bc) return fail(DVM_ERR_ARG, "face must be 0..5");
    if (bc->kind < 0 || bc->kind > 2) return fail(DVM_ERR_ARG, "bad boundary kind");
    if (bc->kind != DVM_BC_SPECULAR && !(bc->T > 0)) return fail(DVM_ERR_ARG, "T must be > 0");
    if (bc->kind == DVM_BC_FREE && !(bc->rho > 0)) return fail(DVM_ERR_ARG, "free-stream rho must be > 0");
    if (bc->kind == DVM_BC_SPECULAR) {
        if (face != 4) return fail(DVM_ERR_ARG, "a specular plane is supported on the z- face only");
        if (c->vg.m[2] % 2) return fail(DVM_ERR_ARG, "a specular plane needs an even velocity count along z");
    }
    c->faces[face] = *bc;
    c->spec_on = c->faces[4].kind == DVM_BC_SPECULAR;
    return DVM_OK;
}

dvm_status dvm_set_solid(dvm_ctx* c, const unsigned char* mask, const double u_wall[3], double T_wall)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (c->bound) return fail(DVM_ERR_STATE, "the solid must be set before binding the workspace");
    if (!mask) {
        c->solid.clear();
        return DVM_OK;
    }
    if (!(T_wall > 0)) return fail(DVM_ERR_ARG, "T_wall must be > 0");
    c->solid.assign(mask, mask + c->N);
    if (u_wall) for (int d = 0; d < 3; ++d) c->solid_u[d] = u_wall[d];
    c->solid_T = T_wall;
    return DVM_OK;
}

dvm_status dvm_set_spacing(dvm_ctx* c, const double* hx, const double* hy, const double* hz)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (c->bound) return fail(DVM_ERR_STATE, "cell sizes must be set before binding the workspace");
    const double* in[3] = {hx, hy, hz};
    const int n3[3] = {c->g.nx, c->g.ny, c->g.nz};
    const double L3[3] = {c->g.lx, c->g.ly, c->g.lz};
    for (int d = 0; d < 3; ++d) {
        if (!in[d]) continue;
        double sum = 0;
        for (int i = 0; i < n3[d]; ++i) {
            if (!(in[d][i] > 0) || !isfinite(in[d][i])) return fail(DVM_ERR_ARG, "axis %d: cell size %d must be > 0", d, i);
            sum += in[d][i];
        }
        if (fabs(sum - L3[d]) > 1e-9 * L3[d]) return fail(DVM_ERR_ARG, "axis %d: cell sizes sum to %.17g, not the length %.17g", d, sum, L3[d]);
    }
    bool any = false;
    std::vector<double> old_h[3] = {c->h[0], c->h[1], c->h[2]};
    const bool old_nu = c->nonuniform;
    for (int d = 0; d < 3; ++d) {
        if (in[d]) {
            c->h[d].assign(in[d], in[d] + n3[d]);
            any = true;
        } else {
            c->h[d].assign(n3[d], c->dx[d]);
        }
    }
    c->nonuniform = any;
    derive_schedule(c);
    if (any && c->model == 1 && c->VL < 2) {
        for (int d = 0; d < 3; ++d) c->h[d] = old_h[d];
        c->nonuniform = old_nu;
        derive_schedule(c);
        return fail(DVM_ERR_ARG, "ES-BGK on a stretched mesh takes the pipelined sweep with 2 or more velocities "
                    "per lane, which this velocity set does not fill (the mesh is left as it was)");
    }
    return DVM_OK;
}

dvm_status dvm_set_velocity_axes(dvm_ctx* c, const double* xi_x, const double* w_x, const double* xi_y,
                                 const double* w_y, const double* xi_z, const double* w_z)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (c->bound) return fail(DVM_ERR_STATE, "velocity axes must be set before binding the workspace");
    const double* xs[3] = {xi_x, xi_y, xi_z};
    const double* ws[3] = {w_x, w_y, w_z};
    for (int d = 0; d < 3; ++d) {
        if (!xs[d] != !ws[d]) return fail(DVM_ERR_ARG, "axis %d: give both nodes and weights, or neither", d);
        if (!xs[d]) continue;
        const int M = c->vg.m[d];
        double big = 0;
        for (int a = 0; a < M; ++a) big = fmax(big, fabs(xs[d][a]));
        for (int a = 0; a < M; ++a) {
            if (!isfinite(xs[d][a]) || !(ws[d][a] > 0) || !isfinite(ws[d][a]))
                return fail(DVM_ERR_ARG, "axis %d: node %d or its weight is invalid", d, a);
            if (a > 0 && !(xs[d][a] > xs[d][a - 1])) return fail(DVM_ERR_ARG, "axis %d: nodes must increase", d);
            if (fabs(xs[d][a] + xs[d][M - 1 - a]) > 1e-12 * big || fabs(ws[d][a] - ws[d][M - 1 - a]) > 1e-12 * ws[d][a])
                return fail(DVM_ERR_ARG, "axis %d: nodes and weights must be symmetric about 0", d);
        }
    }
    for (int d = 0; d < 3; ++d) {
        if (xs[d]) {
            c->vnode[d].assign(xs[d], xs[d] + c->vg.m[d]);
            c->vweight[d].assign(ws[d], ws[d] + c->vg.m[d]);
        } else {
            c->vnode[d].clear();
            c->vweight[d].clear();
        }
    }
    return DVM_OK;
}

dvm_status dvm_set_model(dvm_ctx* c, int model)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (c->bound) return fail(DVM_ERR_STATE, "the model must be set before binding the workspace");
    if (model != 0 && model != 1) return fail(DVM_ERR_ARG, "model must be 0 (Shakhov) or 1 (ES-BGK), got %d", model);
    if (model == 1 && !(c->gas.pr >= 2.0 / 3.0 - 1e-12))
        return fail(DVM_ERR_ARG, "ES-BGK needs Pr >= 2/3 (a positive-definite Gaussian), got %g", c->gas.pr);
    const int old = c->model;
    c->model = model;
    derive_schedule(c);
    if (model == 1 && c->nonuniform && c->VL < 2) {
        c->model = old;
        derive_schedule(c);
        return fail(DVM_ERR_ARG, "ES-BGK on a stretched mesh takes the pipelined sweep with 2 or more velocities "
                    "per lane, which this velocity set does not fill");
    }
    return DVM_OK;
}

dvm_status dvm_get_stress(dvm_ctx* c, double* P)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (c->model != 1) return fail(DVM_ERR_STATE, "the stress is kept for the ES-BGK model only");
    if (!c->initialized) return fail(DVM_ERR_STATE, "no state yet");
    if (!P) return fail(DVM_ERR_ARG, "NULL");
    if (dvm_status e = check_workspace_owner(c)) return e;
    const size_t N = c->N;
    HIPCHK(hipMemcpyAsync(P, c->P<double>(c->off.stress) + (size_t)c->cur * 6 * N, sizeof(double) * 6 * N,
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DVM_OK;
}

dvm_status dvm_set_stress(dvm_ctx* c, const double* P)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (c->model != 1) return fail(DVM_ERR_STATE, "the stress is kept for the ES-BGK model only");
    if (!c->initialized) return fail(DVM_ERR_STATE, "set a state first");
    if (!P) return fail(DVM_ERR_ARG, "NULL");
    if (dvm_status e = check_workspace_owner(c)) return e;
    const size_t N = c->N;
    for (size_t i = 0; i < 6 * N; ++i)
        if (!isfinite(P[i])) return fail(DVM_ERR_ARG, "stress value %zu is not finite", i);
    HIPCHK(hipMemcpyAsync(c->P<double>(c->off.stress) + (size_t)c->cur * 6 * N, P, sizeof(double) * 6 * N,
                          hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DVM_OK;
}

dvm_status dvm_set_order(dvm_ctx* c, int order)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (c->bound) return fail(DVM_ERR_STATE, "the order must be set before binding the workspace");
    if (order != 1 && order != 2) return fail(DVM_ERR_ARG, "order must be 1 or 2 (got %d)", order);
    c->order = order;
    derive_schedule(c);
    return DVM_OK;
}

dvm_status dvm_set_parameter_precision(dvm_ctx* c, int bits)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (c->bound) return fail(DVM_ERR_STATE, "the parameter precision must be set before binding the workspace");
    if (bits != 32 && bits != 64) return fail(DVM_ERR_ARG, "bits must be 32 or 64 (got %d)", bits);
    if (c->prec == DVM_F64) {
        if (bits == 32) return fail(DVM_ERR_ARG, "an FP64 context keeps its parameters in FP64");
        return DVM_OK;
    }
    c->wide = bits == 64;
    return DVM_OK;
}

dvm_status dvm_set_schedule(dvm_ctx* c, int vel_per_lane, int bx, int by, int bz, int body)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (c->bound) return fail(DVM_ERR_STATE, "the schedule must be set before binding the workspace");
    if (vel_per_lane < 0 || vel_per_lane > 8 || bx < 0 || bx > 8 || by < 0 || by > 8 || bz < 0 || bz > 256 ||
        body < 0 || body > 3)
        return fail(DVM_ERR_ARG, "schedule out of range (vel_per_lane %d, brick %dx%dx%d, body %d)", vel_per_lane,
                    bx, by, bz, body);
    const int old[5] = {c->req_vl, c->req_bx, c->req_by, c->req_bz, c->req_body};
    c->req_vl = vel_per_lane;
    c->req_bx = bx;
    c->req_by = by;
    c->req_bz = bz;
    c->req_body = body;
    derive_schedule(c);
    if (!c->req_ok) {
        c->req_vl = old[0];
        c->req_bx = old[1];
        c->req_by = old[2];
        c->req_bz = old[3];
        c->req_body = old[4];
        derive_schedule(c);
        return fail(DVM_ERR_ARG, "no sweep kernel with %d velocities per lane, %dx%d bricks and body %d is built for "
                    "this precision, mesh kind, order and model", vel_per_lane, bx, by, body);
    }
    return DVM_OK;
}

dvm_status dvm_set_solid_mask(dvm_ctx* c, const unsigned char* mask, const double u_wall[3], double T_wall)
{
    return dvm_set_solid(c, mask, u_wall, T_wall);
}

dvm_status dvm_set_sweep_streams(dvm_ctx* c, int streams)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (streams != 1 && streams != 2 && streams != 4 && streams != 8)
        return fail(DVM_ERR_ARG, "streams must be 1, 2, 4 or 8 (got %d)", streams);
    if (c->fork_ev && streams > c->nstreams)
        return fail(DVM_ERR_STATE, "the sweep streams are created; more cannot be added");
    c->nstreams = streams;
    return DVM_OK;
}

dvm_status dvm_set_velocity_groups(dvm_ctx* c, int groups)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (c->bound) return fail(DVM_ERR_STATE, "velocity groups must be set before binding the workspace");
    if (groups < 1) return fail(DVM_ERR_ARG, "groups must be >= 1 (got %d)", groups);
    c->groups_req = groups;
    derive_schedule(c);
    return DVM_OK;
}

dvm_status dvm_set_closed(dvm_ctx* c, int closed)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    c->closed = closed ? 1 : 0;
    return DVM_OK;
}

dvm_status dvm_required_workspace(dvm_ctx* c, size_t* bytes)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (!bytes) return fail(DVM_ERR_ARG, "bytes is NULL");
    layout(c);
    *bytes = c->off.end;
    return DVM_OK;
}

namespace {

// checks that need no workspace: the schedule has a kernel and fits
dvm_status check_bindable(dvm_ctx* c)
{
    if (c->bound) return fail(DVM_ERR_STATE, "workspace already bound");
    if (!c->req_ok)
        return fail(DVM_ERR_ARG, "the schedule set with dvm_set_schedule has no kernel for the order, model or "
                    "mesh kind set after it");
    if (!c->fits32)
        return fail(DVM_ERR_ARG, "a face row of this grid and velocity set exceeds the 32-bit offsets of the "
                    "sweep even with one-cell brick columns: use more velocity groups");
    if (!sweep_variant_available(c->prec, c->VL, c->BX, c->BY, c->nonuniform, c->order == 2, c->model == 1) ||
        ((c->order == 2 || c->model == 1) && c->nonuniform && c->PF != 1) ||
        ((c->order == 2 || c->model == 1) && c->BX == 3 && c->PF != 1))
        return fail(DVM_ERR_ARG, "no sweep kernel is built for %d velocities per lane, %dx%d bricks and body %d with "
                    "this precision, mesh kind, order and model (a stretched mesh at second order or with ES-BGK, "
                    "and 3x2 bricks at second order or with ES-BGK, take the pipelined body with 2 or more "
                    "velocities per lane)", c->VL, c->BX, c->BY, c->PF + 1);
    if (c->wide && (c->PF == 0 || !sweep_wide_params_available(c->prec, c->VL, c->BX, c->BY, c->nonuniform,
                                                                c->order == 2, c->model == 1)))
        return fail(DVM_ERR_ARG, "FP64 parameters beside FP32 storage are built for the first-order Shakhov sweep "
                    "on a uniform mesh with 4 velocities per lane, 4x2 bricks and a pipelined body only");
    layout(c);
    return DVM_OK;
}

// carve the workspace, upload the tables, compute the emission shapes; every
// buffer a kernel reads before writing it is written here or by the initial
// state, so the workspace's previous contents do not matter
dvm_status bind_impl(dvm_ctx* c, void* ptr, size_t bytes)
{
    c->ws = (char*)ptr;
    c->ws_bytes = bytes;
    hipStream_t st = c->stream;

    // velocity axes: uniform (exactly antisymmetric nodes) with trapezoid
    // weights, or the nodes and weights given to dvm_set_velocity_axes
    std::vector<double> axes((2 * 3 + 5) * MAXM, 0.0);
    std::vector<double> xi[3];
    for (int d = 0; d < 3; ++d) {
        const int M = c->vg.m[d];
        const double V = c->vg.vmax[d];
        const double half = V / (M - 1), h = 2.0 * V / (M - 1);
        xi[d].resize(M);
        for (int a = 0; a < M; ++a) {
            const bool given = !c->vnode[d].empty();
            xi[d][a] = given ? c->vnode[d][a] : (double)(2 * a - (M - 1)) * half;
            axes[d * MAXM + a] = xi[d][a];
            axes[3 * MAXM + d * MAXM + a] = given ? c->vweight[d][a] : (a == 0 || a == M - 1) ? 0.5 * h : h;
        }
    }
    // the x axis's w xi^p, p = 0..4, five per node
    for (int a = 0; a < c->vg.m[0]; ++a) {
        double t = axes[3 * MAXM + a];
        for (int p = 0; p < 5; ++p, t *= xi[0][a]) axes[6 * MAXM + 5 * a + p] = t;
    }
    build_cellinfo(c);
    std::vector<double> lt = build_lanetab(c, xi);
    std::vector<double> ks(4 * NKIND, 0.0);
    for (int k = 0; k < NKIND; ++k) {
        const double* u = k < 6 ? c->faces[k].u : c->solid_u;
        double T = k < 6 ? c->faces[k].T : c->solid_T;
        if (!(T > 0)) T = 1.0;
        ks[4 * k + 0] = u[0];
        ks[4 * k + 1] = u[1];
        ks[4 * k + 2] = u[2];
        ks[4 * k + 3] = T;
    }
    HIPCHK(hipMemcpyAsync(c->ws + c->off.axes, axes.data(), sizeof(double) * axes.size(), hipMemcpyHostToDevice, st));
    {
        std::vector<double> hs;
        const int n3[3] = {c->g.nx, c->g.ny, c->g.nz};
        for (int d = 0; d < 3; ++d)
            for (int i = 0; i < n3[d]; ++i) hs.push_back(cell_size(c, d, i));
        c->hstage = hs;
        HIPCHK(hipMemcpyAsync(c->ws + c->off.spacing, c->hstage.data(), sizeof(double) * c->hstage.size(),
                              hipMemcpyHostToDevice, st));
    }
    HIPCHK(hipMemcpyAsync(c->ws + c->off.cellinfo, c->cellinfo.data(), sizeof(uint32_t) * c->N, hipMemcpyHostToDevice, st));
    if (c->order == 2 && c->nonuniform) {
        // the weight of a cell's own slope in the value it carries through
        // its downstream face: the straight line through its centre and its
        // upwind neighbour's, at the face, is f + theta (f - f_up) with
        // theta = h / (h + h_up); per axis, the + direction (upwind i - 1)
        // then the - direction (upwind i + 1); 1/2 where the upwind side is
        // the box (a symmetry plane's mirror cell has the cell's own size)
        std::vector<double>& th = c->thstage;
        th.clear();
        const int n3[3] = {c->g.nx, c->g.ny, c->g.nz};
        for (int d = 0; d < 3; ++d)
            for (int dir = 0; dir < 2; ++dir)
                for (int i = 0; i < n3[d]; ++i) {
                    const int up = dir == 0 ? i - 1 : i + 1;
                    const double h = cell_size(c, d, i);
                    th.push_back(up < 0 || up >= n3[d] ? 0.5 : h / (h + cell_size(c, d, up)));
                }
        HIPCHK(hipMemcpyAsync(c->ws + c->off.theta, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice,
                              st));
    }
    HIPCHK(hipMemcpyAsync(c->ws + c->off.bricks, c->bricks.data(), sizeof(int) * c->bricks.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(c->ws + c->off.lanetab, lt.data(), sizeof(double) * lt.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(c->ws + c->off.kstate, ks.data(), sizeof(double) * ks.size(), hipMemcpyHostToDevice, st));
    // partial slots of tiles that an octant does not have stay zero
    HIPCHK(hipMemsetAsync(c->ws + c->off.partial, 0, c->off.xface - c->off.partial, st));
    // dependency-driven sweep: no brick ready, counter at zero
    if (c->PF == 2) HIPCHK(hipMemsetAsync(c->ws + c->off.ready, 0, c->off.end - c->off.ready, st));
    c->epoch = 0;
    c->qbase = 0;
    const Consts C = make_consts(c);
    const DevPtrs D = make_ptrs(c);
    HIPCHK(launch_emission(C, D, c->P<double>(c->off.kstate), NKIND, c->ws + c->off.ghat,
                           c->P<double>(c->off.ghat64), c->P<double>(c->off.gout), c->prec, st));
    HIPCHK(hipStreamSynchronize(st));
    c->bound = true;
    c->initialized = false;
    return DVM_OK;
}

}  // namespace

dvm_status dvm_bind_workspace(dvm_ctx* c, void* ptr, size_t bytes)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (!ptr) return fail(DVM_ERR_ARG, "workspace pointer is NULL");
    if ((uintptr_t)ptr & 255) return fail(DVM_ERR_ARG, "workspace must be 256-byte aligned");
    if (dvm_status e = check_bindable(c)) return e;
    if (bytes < c->off.end) return fail(DVM_ERR_OOM, "workspace too small: %zu < %zu bytes", bytes, c->off.end);
    return bind_impl(c, ptr, bytes);
}

dvm_status dvm_bind_static_workspace(dvm_ctx* c)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (dvm_status e = check_bindable(c)) return e;
    if (c->off.end > kStaticWorkspaceBytes)
        return fail(DVM_ERR_OOM, "the context needs %zu bytes of workspace, more than the %zu bytes of the static "
                    "workspace: lend one with dvm_bind_workspace", c->off.end, kStaticWorkspaceBytes);
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(DVM_ERR_DEVICE, "device %d out of range", dev);
    if (c->stream) {
        hipDevice_t sdev = -1;
        HIPCHK(hipStreamGetDevice(c->stream, &sdev));
        if (sdev != dev)
            return fail(DVM_ERR_ARG, "the context's stream is on device %d, the current device is %d", (int)sdev,
                        dev);
    }
    void* p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (!g_static_ptr[dev]) {
            void* a = nullptr;
            const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !a)
                return fail(DVM_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                            hipGetErrorString(e));
            g_static_ptr[dev] = a;
        }
        p = g_static_ptr[dev];
        // the previous owner loses the workspace before it is overwritten
        g_static_owner[dev] = c;
    }
    c->static_dev = dev;
    const dvm_status st = bind_impl(c, p, kStaticWorkspaceBytes);
    if (st != DVM_OK) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_owner[dev] == c) g_static_owner[dev] = nullptr;
        c->static_dev = -1;
        c->ws = nullptr;
    }
    return st;
}

dvm_status dvm_init_fields(dvm_ctx* c, const double* rho, const double* u, const double* T, double target_mass)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (!c->bound) return fail(DVM_ERR_STATE, "bind a workspace first");
    if (!rho || !u || !T) return fail(DVM_ERR_ARG, "NULL field");
    if (dvm_status e = check_workspace_owner(c)) return e;
    const size_t N = c->N;
    double mass = 0;
    for (size_t i = 0; i < N; ++i) {
        if (c->cellinfo[i] & SOLID_BIT) continue;
        if (!(rho[i] > 0) || !(T[i] > 0) || !isfinite(rho[i]) || !isfinite(T[i]) || !isfinite(u[i]) ||
            !isfinite(u[N + i]) || !isfinite(u[2 * N + i]))
            return fail(DVM_ERR_NONPHYSICAL, "cell %zu: rho, T must be > 0 and finite", i);
        mass += rho[i] * cell_volume(c, i);
    }
    const double scale = target_mass > 0 ? target_mass / mass : 1.0;
    std::vector<double> Wh(5 * N, 0.0);
    for (size_t i = 0; i < N; ++i) {
        if (c->cellinfo[i] & SOLID_BIT) continue;
        const double r = rho[i] * scale;
        const double ux = u[i], uy = u[N + i], uz = u[2 * N + i];
        Wh[i] = r;
        Wh[N + i] = r * ux;
        Wh[2 * N + i] = r * uy;
        Wh[3 * N + i] = r * uz;
        Wh[4 * N + i] = 0.5 * r * (ux * ux + uy * uy + uz * uz) + 0.75 * r * T[i];
    }
    return upload_initial(c, Wh);
}

dvm_status dvm_init_uniform(dvm_ctx* c, double rho, const double u[3], double T)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (!c->bound) return fail(DVM_ERR_STATE, "bind a workspace first");
    if (!u) return fail(DVM_ERR_ARG, "u is NULL");
    const size_t N = c->N;
    std::vector<double> r(N, rho), uu(3 * N), t(N, T);
    for (size_t i = 0; i < N; ++i) {
        uu[i] = u[0];
        uu[N + i] = u[1];
        uu[2 * N + i] = u[2];
    }
    return dvm_init_fields(c, r.data(), uu.data(), t.data(), 0.0);
}

dvm_status dvm_iterate(dvm_ctx* c, int max_iters, double tol, int* iters_done, double* residual)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (!c->initialized) return fail(DVM_ERR_STATE, "initialise the state first");
    if (max_iters < 0) return fail(DVM_ERR_ARG, "max_iters must be >= 0");
    if (dvm_status e = check_workspace_owner(c)) return e;
    if (iters_done) *iters_done = 0;
    double hout[8];
    double r = INFINITY;
    for (int it = 0; it < max_iters; ++it) {
        const dvm_status st = run_iteration(c, hout);
        if (st != DVM_OK) return st;
        const int flag = (int)hout[6];
        if (flag & 8)
            return fail(DVM_ERR_DEVICE, "iteration %d: a sweep work unit waited too long for its upwind bricks; "
                        "the iterate is not updated", it + 1);
        bool finite = true;
        for (int v = 0; v < 5; ++v) finite = finite && isfinite(hout[v]);
        if (flag || !finite) {
            if (residual) *residual = r;
            return fail(DVM_ERR_NONPHYSICAL, "non-physical state in iteration %d (flag %d); kept the last good iterate",
                        it + 1, flag);
        }
        c->cur = 1 - c->cur;
        r = 0;
        for (int v = 0; v < 5; ++v) {
            c->res[v] = hout[v];
            if (hout[v] > r) r = hout[v];
        }
        if (iters_done) *iters_done = it + 1;
        if (residual) *residual = r;
        if (tol > 0 && r <= tol) return DVM_OK;
    }
    if (tol > 0 && max_iters > 0) return DVM_NOT_CONVERGED;
    return DVM_OK;
}

dvm_status dvm_get_residuals(dvm_ctx* c, double r[5])
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (!r) return fail(DVM_ERR_ARG, "NULL");
    for (int v = 0; v < 5; ++v) r[v] = c->res[v];
    return DVM_OK;
}

dvm_status dvm_get_state(dvm_ctx* c, double* W, double* q, double* rho_w, double* M0)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (!c->initialized) return fail(DVM_ERR_STATE, "no state yet");
    if (dvm_status e = check_workspace_owner(c)) return e;
    const size_t N = c->N;
    hipStream_t st = c->stream;
    if (W) HIPCHK(hipMemcpyAsync(W, c->P<double>(c->off.W) + c->cur * 5 * N, sizeof(double) * 5 * N, hipMemcpyDeviceToHost, st));
    if (q) HIPCHK(hipMemcpyAsync(q, c->P<double>(c->off.q) + c->cur * 3 * N, sizeof(double) * 3 * N, hipMemcpyDeviceToHost, st));
    if (rho_w) HIPCHK(hipMemcpyAsync(rho_w, c->P<double>(c->off.rw) + c->cur * 6 * N, sizeof(double) * 6 * N, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (M0) *M0 = c->M0;
    return DVM_OK;
}

dvm_status dvm_set_state(dvm_ctx* c, const double* W, const double* q, const double* rho_w, double M0)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (!c->bound) return fail(DVM_ERR_STATE, "bind a workspace first");
    if (!W || !q || !rho_w) return fail(DVM_ERR_ARG, "NULL");
    if (dvm_status e = check_workspace_owner(c)) return e;
    const size_t N = c->N;
    for (size_t i = 0; i < N; ++i) {
        if (c->cellinfo[i] & SOLID_BIT) continue;
        if (!(W[i] > 0) || !isfinite(W[i])) return fail(DVM_ERR_NONPHYSICAL, "cell %zu: rho must be > 0", i);
    }
    hipStream_t st = c->stream;
    c->cur = 0;
    HIPCHK(hipMemcpyAsync(c->P<double>(c->off.W), W, sizeof(double) * 5 * N, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(c->P<double>(c->off.q), q, sizeof(double) * 3 * N, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(c->P<double>(c->off.rw), rho_w, sizeof(double) * 6 * N, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    // ES-BGK: the stress restarts at the equilibrium of the given state
    if (upload_equilibrium_stress(c, W)) return DVM_ERR_DEVICE;
    c->M0 = M0;
    c->initialized = true;
    for (int v = 0; v < 5; ++v) c->res[v] = 0;
    return DVM_OK;
}

dvm_status dvm_get_fields(dvm_ctx* c, double* rho, double* u, double* T, double* q)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (!c->initialized) return fail(DVM_ERR_STATE, "no state yet");
    const size_t N = c->N;
    std::vector<double> W(5 * N), qq(3 * N);
    dvm_status st = dvm_get_state(c, W.data(), qq.data(), nullptr, nullptr);
    if (st) return st;
    for (size_t i = 0; i < N; ++i) {
        const bool sol = (c->cellinfo[i] & SOLID_BIT) != 0;
        const double r = sol ? 0.0 : W[i];
        double U[3] = {0, 0, 0}, t = 0;
        if (!sol) {
            for (int d = 0; d < 3; ++d) U[d] = W[(d + 1) * N + i] / r;
            t = (W[4 * N + i] - 0.5 * r * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2])) / (0.75 * r);
        }
        if (rho) rho[i] = r;
        if (T) T[i] = t;
        if (u) for (int d = 0; d < 3; ++d) u[d * N + i] = U[d];
        if (q) for (int d = 0; d < 3; ++d) q[d * N + i] = sol ? 0.0 : qq[d * N + i];
    }
    return DVM_OK;
}

dvm_status dvm_get_info(dvm_ctx* c, dvm_info* info)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (!info) return fail(DVM_ERR_ARG, "NULL");
    layout(c);
    int nfluid = c->N;
    if (!c->solid.empty()) {
        nfluid = 0;
        for (uint8_t s : c->solid) nfluid += s ? 0 : 1;
    }
    info->nx = c->g.nx;
    info->ny = c->g.ny;
    info->nz = c->g.nz;
    info->ncells = c->N;
    info->nfluid = nfluid;
    for (int d = 0; d < 3; ++d) info->m[d] = c->vg.m[d];
    info->nvel = c->NV;
    info->precision = c->prec;
    info->brick[0] = c->BX;
    info->brick[1] = c->BY;
    info->brick[2] = c->BZ;
    info->vel_per_lane = c->VL;
    info->tiles_per_octant = c->ntiles;
    int launches = 0;
    for (int T = 0; T < c->ndiag; ++T) launches += c->diag_cnt[T] > 0;
    const int ns = c->PF == 2 ? 1 : std::min(c->nstreams, c->spec_on ? 4 : 8);
    info->sweep_launches = (c->PF == 2 ? 1 : launches) * (c->spec_on ? 2 : 1) * c->ngroups * ns;
    info->workspace_bytes = c->off.end;
    info->pipelined = c->PF;
    info->velocity_groups = c->ngroups;
    info->parameter_bits = c->pprec() == DVM_F64 ? 64 : 32;
    info->sweep_streams = ns;
    return DVM_OK;
}

dvm_status dvm_set_timing(dvm_ctx* c, int enable)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (enable < 0 || enable > 2) return fail(DVM_ERR_ARG, "timing level must be 0, 1 or 2 (got %d)", enable);
    if (enable && !c->ev[0])
        for (int k = 0; k < 4; ++k) HIPCHK(hipEventCreate(&c->ev[k]));
    c->timing = enable;
    c->t_params = c->t_sweep = c->t_final = 0;
    c->t_iters = 0;
    c->t_launch = 0;
    c->n_launch = 0;
    return DVM_OK;
}

dvm_status dvm_get_launch_timings(dvm_ctx* c, double* ms_total, long long* launches)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (ms_total) *ms_total = c->t_launch;
    if (launches) *launches = c->n_launch;
    c->t_launch = 0;
    c->n_launch = 0;
    return DVM_OK;
}

dvm_status dvm_get_timings(dvm_ctx* c, double* ms_params, double* ms_sweep, double* ms_finalize, int* iterations)
{
    if (check_ctx(c)) return DVM_ERR_ARG;
    if (ms_params) *ms_params = c->t_params;
    if (ms_sweep) *ms_sweep = c->t_sweep;
    if (ms_finalize) *ms_finalize = c->t_final;
    if (iterations) *iterations = c->t_iters;
    c->t_params = c->t_sweep = c->t_final = 0;
    c->t_iters = 0;
    return DVM_OK;
}

dvm_status dvm_selftest_wave_reduce(const double* in, double* out)
{
    if (!in || !out) return fail(DVM_ERR_ARG, "NULL");
    double *din = nullptr, *dout = nullptr;
    HIPCHK(hipMalloc(&din, sizeof(double) * 64 * 13));
    HIPCHK(hipMalloc(&dout, sizeof(double) * 13));
    HIPCHK(hipMemcpy(din, in, sizeof(double) * 64 * 13, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(dout, 0, sizeof(double) * 13));
    HIPCHK(launch_selftest_reduce(din, dout, nullptr));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(out, dout, sizeof(double) * 13, hipMemcpyDeviceToHost));
    HIPCHK(hipFree(din));
    HIPCHK(hipFree(dout));
    return DVM_OK;
}

void dvm_destroy(dvm_ctx* c)
{
    if (!c) return;
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_owner[c->static_dev] == c) g_static_owner[c->static_dev] = nullptr;
    }
    for (int k = 0; k < 4; ++k)
        if (c->ev[k]) (void)hipEventDestroy(c->ev[k]);
    for (hipEvent_t e : c->lev) (void)hipEventDestroy(e);
    for (int k = 0; k < 8; ++k) {
        if (c->sub[k]) (void)hipStreamDestroy(c->sub[k]);
        if (c->join_ev[k]) (void)hipEventDestroy(c->join_ev[k]);
    }
    if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
    delete c;
}

}  // extern "C"
